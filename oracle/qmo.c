/*
 * qmo.c -- ORACLE for the round-based constrained Delaunay refinement loop.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential CPU statement
 * of what the GPU library computes; only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * GPU library.
 *
 * What it computes (paper, Section 2 "Our Proposed Algorithm", with the data
 * model of Section 1): elements -- subsegments, subfaces and bad tetrahedra --
 * are split in that order, in rounds, until no element is left to split.  In
 * one round:
 *
 *   1. classify   every element; the round class is the first of
 *                 subsegment / subface / tetrahedron that has candidates;
 *   2. split      each candidate gets its splitting point (midpoint,
 *                 circumcircle centre, circumsphere centre) and a fixed
 *                 pseudo-random priority (the paper's predetermined
 *                 priorities);
 *   3. locate     the element holding the point (walk), Section 2 grow step;
 *   4. grow       the Delaunay region: subfaces whose circumcircle and tets
 *                 whose circumsphere strictly enclose the point, connected to
 *                 the seed;
 *   5. validate   filter points that would create short edges or break the
 *                 mesh (the paper's filtering of splitting points);
 *   6. select     keep a maximal set of points whose regions (with their
 *                 face-neighbour ring) are mutually disjoint, greedily by
 *                 priority (the grow-and-blast outcome made deterministic);
 *   7. insert     all kept points; the mesh is again a CDT.
 *
 * Every decision depends only on vertex ids and coordinates, never on array
 * slots.  The readings taken where the paper is silent are spelled out at the
 * functions that implement them.
 *
 * Options set before a run: the sub-phase reading of the class order
 * (qmo_set_subphases), a check of the mesh after every round
 * (qmo_set_round_check), a recorded round (qmo_set_dump_round), forced equal
 * priorities (qmo_set_key_mask), and resuming from a refinement state
 * (qmo_set_resume; every result exports its state, qmo_result_state).
 * qm_oracle_refine takes the GPU library's call layout and return codes, so
 * that a test can hand one marshalled argument set to either engine.
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <time.h>

#include "qmo_exact.h"

/* ----------------------------------------------------------- constants */
enum { CLS_SS = 0, CLS_SF = 1, CLS_TET = 2, CLS_NONE = 3 };
enum { ST_OK = 0, ST_REJECT = 1, ST_EXEMPT = 2 };
enum { EX_NONE = 0, EX_NONFINITE = 1, EX_WALK = 2, EX_ENC_EXEMPT = 3, EX_HMIN = 4,
       EX_RFTET = 5, EX_FACE = 6, EX_EDGE2D = 7, EX_MANIFOLD = 8, EX_DELAUNAY = 9, EX_NREASON = 10 };
#define FL_QUEUED 1
#define FL_EXEMPT 2
#define WALK_CAP 1000000

/* inward face triples: face f is opposite vertex f, and
   orient3d(face[0], face[1], face[2], v_f) > 0 for a positive tet */
static const int FI[4][3] = {{1, 3, 2}, {0, 2, 3}, {0, 3, 1}, {0, 1, 2}};

/* ------------------------------------------------------------- vectors */
typedef struct { int* a; int n, cap; } IV;
static void iv_push(IV* v, int x) {
    if (v->n == v->cap) { v->cap = v->cap ? 2 * v->cap : 16; v->a = (int*)realloc(v->a, sizeof(int) * (size_t)v->cap); }
    v->a[v->n++] = x;
}
static void iv_free(IV* v) { free(v->a); v->a = NULL; v->n = v->cap = 0; }
static int iv_has(const IV* v, int x) { for (int i = 0; i < v->n; ++i) if (v->a[i] == x) return 1; return 0; }

/* ------------------------------------------------------------ hash map */
/* open addressing on sorted id tuples (padded with -1) */
typedef struct { int k[4]; int v[2]; unsigned char st; } HE;
typedef struct { HE* e; size_t cap, used, n; } HMap;

static uint64_t hm_hash(const int* k) {
    uint64_t h = 0x51ED270B27A1F00Dull;
    for (int i = 0; i < 4; ++i) h = qmo_mix64(h ^ (uint64_t)(uint32_t)k[i]);
    return h;
}
static void hm_init(HMap* m, size_t cap) {
    size_t c = 64; while (c < cap) c <<= 1;
    m->e = (HE*)calloc(c, sizeof(HE)); m->cap = c; m->used = m->n = 0;
}
static void hm_free(HMap* m) { free(m->e); m->e = NULL; m->cap = m->used = m->n = 0; }
static HE* hm_get(const HMap* m, const int* k) {
    size_t i = hm_hash(k) & (m->cap - 1);
    for (;;) {
        HE* e = &m->e[i];
        if (e->st == 0) return NULL;
        if (e->st == 1 && !memcmp(e->k, k, sizeof e->k)) return e;
        i = (i + 1) & (m->cap - 1);
    }
}
static HE* hm_put(HMap* m, const int* k);
static void hm_rehash(HMap* m, size_t cap) {
    HMap n; hm_init(&n, cap);
    for (size_t i = 0; i < m->cap; ++i)
        if (m->e[i].st == 1) { HE* d = hm_put(&n, m->e[i].k); d->v[0] = m->e[i].v[0]; d->v[1] = m->e[i].v[1]; }
    free(m->e); *m = n;
}
static HE* hm_put(HMap* m, const int* k) {
    if ((m->used + 1) * 10 > m->cap * 7) hm_rehash(m, (m->n + 1) * 4);
    size_t i = hm_hash(k) & (m->cap - 1);
    HE* tomb = NULL;
    for (;;) {
        HE* e = &m->e[i];
        if (e->st == 0) {
            if (tomb) e = tomb; else m->used++;
            memcpy(e->k, k, sizeof e->k); e->v[0] = e->v[1] = -1; e->st = 1; m->n++;
            return e;
        }
        if (e->st == 2 && !tomb) tomb = e;
        if (e->st == 1 && !memcmp(e->k, k, sizeof e->k)) return e;
        i = (i + 1) & (m->cap - 1);
    }
}
static void hm_del(HMap* m, HE* e) { e->st = 2; m->n--; }

static void key2(int* k, int a, int b) { if (a > b) { int t = a; a = b; b = t; } k[0] = a; k[1] = b; k[2] = k[3] = -1; }
static void key3(int* k, int a, int b, int c) {
    int x[3] = {a, b, c};
    for (int i = 0; i < 3; ++i) for (int j = i + 1; j < 3; ++j) if (x[j] < x[i]) { int t = x[i]; x[i] = x[j]; x[j] = t; }
    k[0] = x[0]; k[1] = x[1]; k[2] = x[2]; k[3] = -1;
}
static void sort4(int* x) {
    for (int i = 0; i < 4; ++i) for (int j = i + 1; j < 4; ++j) if (x[j] < x[i]) { int t = x[i]; x[i] = x[j]; x[j] = t; }
}

/* ---------------------------------------------------------------- mesh */
typedef struct { int v[4]; unsigned char alive, exempt; } OTet;

typedef struct {
    double (*V)[3]; int nv, capv;
    int* vt;                 /* a live tet incident to each vertex */
    OTet* T; int nt, capt;   /* tets; dead ones stay with alive = 0 */
    HMap faces;              /* sorted face triple -> up to two (t<<2|f) */
    HMap sf;                 /* subface triple -> facet id, flags */
    HMap ss;                 /* subsegment pair -> segment id, flags */
    int* faxis; int nfacet;  /* projection axis per facet */
    double B2, hmin2;
    int *inR, *tested, *claimed, *instar; int serial, starserial;   /* per-tet scratch stamps */
} Mesh;

static int face_key(const Mesh* M, int t, int f, int* k) {
    const int* v = M->T[t].v;
    key3(k, v[FI[f][0]], v[FI[f][1]], v[FI[f][2]]);
    return 0;
}

static void grow_tet_arrays(Mesh* M) {
    if (M->nt < M->capt) return;
    int old = M->capt;
    M->capt = M->capt ? 2 * M->capt : 1024;
    M->T = (OTet*)realloc(M->T, sizeof(OTet) * (size_t)M->capt);
    M->inR = (int*)realloc(M->inR, sizeof(int) * (size_t)M->capt);
    M->tested = (int*)realloc(M->tested, sizeof(int) * (size_t)M->capt);
    M->claimed = (int*)realloc(M->claimed, sizeof(int) * (size_t)M->capt);
    M->instar = (int*)realloc(M->instar, sizeof(int) * (size_t)M->capt);
    for (int i = old; i < M->capt; ++i) M->inR[i] = M->tested[i] = M->claimed[i] = M->instar[i] = -1;
}

static int add_tet(Mesh* M, const int* v) {
    grow_tet_arrays(M);
    int t = M->nt++;
    OTet* T = &M->T[t];
    memcpy(T->v, v, sizeof T->v); T->alive = 1; T->exempt = 0;
    for (int f = 0; f < 4; ++f) {
        int k[4]; face_key(M, t, f, k);
        HE* e = hm_put(&M->faces, k);
        if (e->v[0] < 0) e->v[0] = (t << 2) | f;
        else if (e->v[1] < 0) e->v[1] = (t << 2) | f;
        else return -1;                       /* face in three tets */
    }
    for (int i = 0; i < 4; ++i) M->vt[v[i]] = t;
    return t;
}

static void del_tet(Mesh* M, int t) {
    for (int f = 0; f < 4; ++f) {
        int k[4]; face_key(M, t, f, k);
        HE* e = hm_get(&M->faces, k);
        if (!e) continue;
        int me = (t << 2) | f;
        if (e->v[0] == me) { e->v[0] = e->v[1]; e->v[1] = -1; }
        else if (e->v[1] == me) e->v[1] = -1;
        if (e->v[0] < 0) hm_del(&M->faces, e);
    }
    M->T[t].alive = 0;
}

/* neighbour across face f of t as (t'<<2|f'), or -1 on the hull */
static int neighbour(const Mesh* M, int t, int f) {
    int k[4]; face_key(M, t, f, k);
    HE* e = hm_get(&M->faces, k);
    if (!e) return -1;
    int me = (t << 2) | f;
    if (e->v[0] == me) return e->v[1];
    return e->v[0];
}

static int tet_has(const OTet* T, int v) { return T->v[0] == v || T->v[1] == v || T->v[2] == v || T->v[3] == v; }

static HE* get_sf(const Mesh* M, int a, int b, int c) { int k[4]; key3(k, a, b, c); return hm_get(&M->sf, k); }
static HE* get_ss(const Mesh* M, int a, int b) { int k[4]; key2(k, a, b); return hm_get(&M->ss, k); }

/* all live tets containing vertex a (breadth-first over faces through a) */
static void star(const Mesh* Mc, int a, IV* out) {
    Mesh* M = (Mesh*)Mc;
    int s = ++M->starserial;
    out->n = 0;
    int t0 = M->vt[a];
    if (t0 < 0 || !M->T[t0].alive || !tet_has(&M->T[t0], a)) return;
    iv_push(out, t0); M->instar[t0] = s;
    for (int i = 0; i < out->n; ++i) {
        int t = out->a[i];
        for (int f = 0; f < 4; ++f) {
            if (M->T[t].v[f] == a) continue;          /* face opposite a lacks a */
            int nb = neighbour(M, t, f);
            if (nb < 0 || M->instar[nb >> 2] == s) continue;
            M->instar[nb >> 2] = s; iv_push(out, nb >> 2);
        }
    }
}

/* all live tets containing edge ab */
static void edge_tets(const Mesh* M, int a, int b, IV* out) {
    IV s = {0};
    star(M, a, &s);
    out->n = 0;
    for (int i = 0; i < s.n; ++i) if (tet_has(&M->T[s.a[i]], b)) iv_push(out, s.a[i]);
    iv_free(&s);
}

/* subfaces (as sorted triples, flattened) containing edge ab */
static void edge_subfaces(const Mesh* M, int a, int b, IV* out) {
    IV et = {0};
    edge_tets(M, a, b, &et);
    out->n = 0;
    for (int i = 0; i < et.n; ++i) {
        const OTet* T = &M->T[et.a[i]];
        for (int j = 0; j < 4; ++j) {
            int c = T->v[j];
            if (c == a || c == b) continue;
            int k[4]; key3(k, a, b, c);
            if (!hm_get(&M->sf, k)) continue;
            int dup = 0;
            for (int q = 0; q < out->n; q += 3)
                if (out->a[q] == k[0] && out->a[q + 1] == k[1] && out->a[q + 2] == k[2]) dup = 1;
            if (!dup) { iv_push(out, k[0]); iv_push(out, k[1]); iv_push(out, k[2]); }
        }
    }
    iv_free(&et);
}

/* the other subface of facet F containing edge (x,y), or 0 if none */
static int facet_neighbour(const Mesh* M, const int* g, int x, int y, int F, int* out) {
    IV s = {0};
    edge_subfaces(M, x, y, &s);
    int found = 0;
    for (int q = 0; q < s.n; q += 3) {
        const int* h = &s.a[q];
        if (h[0] == g[0] && h[1] == g[1] && h[2] == g[2]) continue;
        HE* e = get_sf(M, h[0], h[1], h[2]);
        if (e->v[0] != F) continue;
        memcpy(out, h, 3 * sizeof(int)); found = 1; break;
    }
    iv_free(&s);
    return found;
}

/* the (one or two) live tets having face abc, as t<<2|f */
static int face_tets(const Mesh* M, int a, int b, int c, int* out) {
    int k[4]; key3(k, a, b, c);
    HE* e = hm_get(&M->faces, k);
    if (!e) return 0;
    int n = 0;
    if (e->v[0] >= 0) out[n++] = e->v[0];
    if (e->v[1] >= 0) out[n++] = e->v[1];
    return n;
}

/* ----------------------------------------------------------- candidates */
typedef struct {
    int cls, tup[4], ntup;
    uint64_t key;
    double p[3];
    int status, reason;
    IV RT;        /* region tets */
    IV RF;        /* region subfaces, flattened sorted triples */
    IV Q;         /* queue targets: (kind, a, b, c) with kind 0 = ss, 1 = sf */
    IV bface;     /* boundary faces t<<2|f */
    IV bedge;     /* 2D boundary edges: (x, y, facet, one-sided) */
    IV claim;     /* claimed tets */
    int kept;
    int slot;     /* TET class: the tet's index (valid within the round) */
} Cand;

static void cand_free(Cand* c) {
    iv_free(&c->RT); iv_free(&c->RF); iv_free(&c->Q); iv_free(&c->bface); iv_free(&c->bedge); iv_free(&c->claim);
}

static int rf_has(const IV* RF, const int* g) {
    for (int q = 0; q < RF->n; q += 3)
        if (RF->a[q] == g[0] && RF->a[q + 1] == g[1] && RF->a[q + 2] == g[2]) return 1;
    return 0;
}

static const double* X(const Mesh* M, int v) { return M->V[v]; }

/* Test hook: keys are ANDed with this mask, so that tests can force equal
   keys and exercise the tie rule (ascending tuple). */
static uint64_t g_key_mask = ~(uint64_t)0;
void qmo_set_key_mask(uint64_t m) { g_key_mask = m; }
static uint64_t cand_key(const Cand* c) { return qmo_key(c->cls, c->tup, c->ntup) & g_key_mask; }

/* ---- Step 2: splitting point and priority ---------------------------- */
static void split_point(const Mesh* M, Cand* c) {
    const int* t = c->tup;
    if (c->cls == CLS_SS) qmo_midpoint(X(M, t[0]), X(M, t[1]), c->p);
    else if (c->cls == CLS_SF) qmo_tri_cc(X(M, t[0]), X(M, t[1]), X(M, t[2]), c->p);
    else { double R2; qmo_tet_cc(X(M, t[0]), X(M, t[1]), X(M, t[2]), X(M, t[3]), c->p, &R2); }
    c->key = cand_key(c);
}

/* queue one element; returns whether it is exempt */
static int add_queue(const Mesh* M, Cand* c, int kind, int a, int b, int d) {
    int k[4];
    HE* e;
    if (kind == 0) { key2(k, a, b); e = hm_get(&M->ss, k); }
    else { key3(k, a, b, d); e = hm_get(&M->sf, k); }
    for (int q = 0; q < c->Q.n; q += 4)
        if (c->Q.a[q] == kind && c->Q.a[q + 1] == k[0] && c->Q.a[q + 2] == k[1] && c->Q.a[q + 3] == k[2]) return 0;
    iv_push(&c->Q, kind); iv_push(&c->Q, k[0]); iv_push(&c->Q, k[1]); iv_push(&c->Q, k[2]);
    return e && (e->v[1] & FL_EXEMPT);
}

/* A rejection queues its targets; when every target is already exempt the
   candidate is exempted instead (so that the round still makes progress). */
static void finish_queue(Mesh* M, Cand* c) {
    int all_exempt = 1;
    for (int q = 0; q < c->Q.n; q += 4) {
        int k[4] = {c->Q.a[q + 1], c->Q.a[q + 2], c->Q.a[q + 3], -1};
        HE* e = c->Q.a[q] == 0 ? hm_get(&M->ss, k) : hm_get(&M->sf, k);
        if (!(e->v[1] & FL_EXEMPT)) all_exempt = 0;
    }
    if (all_exempt) { c->status = ST_EXEMPT; c->reason = EX_ENC_EXEMPT; }
    else c->status = ST_REJECT;
}

/* ---- Step 3: locate ------------------------------------------------- */
/* Tet walk from the bad tet toward p: at each tet the faces are tried in
   ascending order of their opposite vertex id and the first face with p
   strictly on its outer side is crossed.  Crossing a subface (hull faces are
   all subfaces) rejects the point and queues that subface. */
static int walk3d(Mesh* M, Cand* c, int t0, int* out_t) {
    int t = t0;
    for (int step = 0; step < WALK_CAP; ++step) {
        const OTet* T = &M->T[t];
        int ord[4] = {0, 1, 2, 3};
        for (int i = 0; i < 4; ++i) for (int j = i + 1; j < 4; ++j)
            if (T->v[ord[j]] < T->v[ord[i]]) { int x = ord[i]; ord[i] = ord[j]; ord[j] = x; }
        int moved = 0;
        for (int i = 0; i < 4 && !moved; ++i) {
            int f = ord[i];
            int a = T->v[FI[f][0]], b = T->v[FI[f][1]], d = T->v[FI[f][2]];
            if (qmo_orient3d(X(M, a), X(M, b), X(M, d), c->p) >= 0) continue;
            if (get_sf(M, a, b, d)) {
                add_queue(M, c, 1, a, b, d);
                finish_queue(M, c);
                return -1;
            }
            int nb = neighbour(M, t, f);
            if (nb < 0) { c->status = ST_EXEMPT; c->reason = EX_WALK; return -1; }  /* unconstrained hull */
            t = nb >> 2; moved = 1;
        }
        if (!moved) { *out_t = t; return 0; }
    }
    c->status = ST_EXEMPT; c->reason = EX_WALK;
    return -1;
}

/* Subface walk on facet F from subface g toward p, in the facet's 2D
   projection: edges are tried in ascending (sorted-pair) order and the first
   edge with p strictly beyond it is crossed.  Crossing a subsegment rejects
   the point and queues that subsegment. */
static int walk2d(Mesh* M, Cand* c, const int* g0, int* out_g) {
    int g[3] = {g0[0], g0[1], g0[2]};
    HE* e0 = get_sf(M, g[0], g[1], g[2]);
    int F = e0->v[0], ax = M->faxis[F];
    static const int EP[3][3] = {{0, 1, 2}, {0, 2, 1}, {1, 2, 0}};
    for (int step = 0; step < WALK_CAP; ++step) {
        int moved = 0;
        for (int i = 0; i < 3 && !moved; ++i) {
            int x = g[EP[i][0]], y = g[EP[i][1]], z = g[EP[i][2]];
            int oz = qmo_orient2d(ax, X(M, x), X(M, y), X(M, z));
            int op = qmo_orient2d(ax, X(M, x), X(M, y), c->p);
            if (op == 0 || op != -oz) continue;
            if (get_ss(M, x, y)) {
                add_queue(M, c, 0, x, y, -1);
                finish_queue(M, c);
                return -1;
            }
            int h[3];
            if (!facet_neighbour(M, g, x, y, F, h)) { c->status = ST_EXEMPT; c->reason = EX_WALK; return -1; }
            memcpy(g, h, sizeof g); moved = 1;
        }
        if (!moved) { memcpy(out_g, g, sizeof g); return 0; }
    }
    c->status = ST_EXEMPT; c->reason = EX_WALK;
    return -1;
}

/* ---- Step 4: grow ---------------------------------------------------- */
/* R_F: subfaces of the seed facets, connected across edges that are not
   subsegments, whose circumcircle strictly encloses p (Section 2 region
   definition; for an off-plane FP64 point the circle is taken as the
   equatorial ball).  Seeds are always included. */
static void grow_rf(Mesh* M, Cand* c) {
    for (int i = 0; i < c->RF.n; i += 3) {
        int g[3] = {c->RF.a[i], c->RF.a[i + 1], c->RF.a[i + 2]};
        int F = get_sf(M, g[0], g[1], g[2])->v[0];
        static const int EP[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int j = 0; j < 3; ++j) {
            int x = g[EP[j][0]], y = g[EP[j][1]];
            if (get_ss(M, x, y)) continue;
            int h[3];
            if (!facet_neighbour(M, g, x, y, F, h)) continue;
            if (rf_has(&c->RF, h)) continue;
            if (qmo_facedot(X(M, h[0]), X(M, h[1]), X(M, h[2]), c->p) < 0) {
                iv_push(&c->RF, h[0]); iv_push(&c->RF, h[1]); iv_push(&c->RF, h[2]);
            }
        }
    }
}

static int face_is_rf(const Mesh* M, const Cand* c, int t, int f) {
    int k[4]; face_key(M, t, f, k);
    return rf_has(&c->RF, k);
}

/* R_T: tets whose circumsphere strictly encloses p (insphere = 0 counts as
   outside: p is always the newest point), connected to the seeds across
   faces that are not subfaces, or are subfaces of R_F.  Seeds are always
   included. */
static void grow_rt(Mesh* M, Cand* c, int s) {
    for (int i = 0; i < c->RT.n; ++i) {
        int t = c->RT.a[i];
        for (int f = 0; f < 4; ++f) {
            int k[4]; face_key(M, t, f, k);
            if (hm_get(&M->sf, k) && !rf_has(&c->RF, k)) continue;
            int nb = neighbour(M, t, f);
            if (nb < 0) continue;
            int n = nb >> 2;
            if (M->tested[n] == s) continue;
            M->tested[n] = s;
            const int* v = M->T[n].v;
            if (qmo_insphere(X(M, v[0]), X(M, v[1]), X(M, v[2]), X(M, v[3]), c->p) > 0) {
                M->inR[n] = s; iv_push(&c->RT, n);
            }
        }
    }
}

static void add_seed_tet(Mesh* M, Cand* c, int t, int s) {
    if (M->inR[t] == s) return;
    M->inR[t] = s; M->tested[t] = s; iv_push(&c->RT, t);
}

/* ---- Step 5: validate ------------------------------------------------- */
static const int EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

/* number of boundary faces containing edge xy */
static int count_bfaces(const Mesh* M, const Cand* c, int x, int y) {
    int cnt = 0;
    for (int q = 0; q < c->bface.n; ++q) {
        const int* w = M->T[c->bface.a[q] >> 2].v;
        int g = c->bface.a[q] & 3;
        int hx = 0, hy = 0;
        for (int r = 0; r < 3; ++r) { hx |= w[FI[g][r]] == x; hy |= w[FI[g][r]] == y; }
        cnt += hx && hy;
    }
    return cnt;
}
/* whether xy is a 2D boundary edge (the new face (x, y, p) is a subface) */
static int is_bedge(const Cand* c, int x, int y) {
    if (x > y) { int t = x; x = y; y = t; }
    for (int q = 0; q < c->bedge.n; q += 4)
        if (c->bedge.a[q] == x && c->bedge.a[q + 1] == y) return 1;
    return 0;
}
/* 1 for a one-sided 2D boundary edge, else 2 */
static int want_bfaces(const Cand* c, int x, int y) {
    if (x > y) { int t = x; x = y; y = t; }
    for (int q = 0; q < c->bedge.n; q += 4)
        if (c->bedge.a[q] == x && c->bedge.a[q + 1] == y && c->bedge.a[q + 3]) return 1;
    return 2;
}

static void validate(Mesh* M, Cand* c, int s) {
    const double* p = c->p;
    /* (a) encroachment: a tet point is rejected when it encroaches a
       subsegment or subface of its region, a subface point when it
       encroaches a subsegment of its region; subsegment points are never
       rejected (Shewchuk's rule, the paper's filtering) */
    if (c->cls != CLS_SS) {
        for (int i = 0; i < c->RT.n; ++i) {
            const OTet* T = &M->T[c->RT.a[i]];
            for (int e = 0; e < 6; ++e) {
                int a = T->v[EDGE[e][0]], b = T->v[EDGE[e][1]];
                if (!get_ss(M, a, b)) continue;
                if (qmo_segdot(X(M, a), X(M, b), p) < 0) add_queue(M, c, 0, a, b, -1);
            }
            if (c->cls == CLS_TET) {
                for (int f = 0; f < 4; ++f) {
                    int a = T->v[FI[f][0]], b = T->v[FI[f][1]], d = T->v[FI[f][2]];
                    if (!get_sf(M, a, b, d)) continue;
                    if (qmo_facedot(X(M, a), X(M, b), X(M, d), p) < 0) add_queue(M, c, 1, a, b, d);
                }
            }
        }
        if (c->Q.n) { finish_queue(M, c); return; }
    }
    /* (b) insertion radius: distance to the nearest region vertex must reach
       h_min (the reading of the paper's short-edge filter) */
    double r2 = INFINITY;
    for (int i = 0; i < c->RT.n; ++i)
        for (int k = 0; k < 4; ++k) { double d2 = qmo_d2(X(M, M->T[c->RT.a[i]].v[k]), p); if (d2 < r2) r2 = d2; }
    for (int i = 0; i < c->RF.n; ++i) { double d2 = qmo_d2(X(M, c->RF.a[i]), p); if (d2 < r2) r2 = d2; }
    if (r2 < M->hmin2) { c->status = ST_EXEMPT; c->reason = EX_HMIN; return; }
    /* (c) every tet on a region subface is a region tet */
    for (int i = 0; i < c->RF.n; i += 3) {
        int tf[2], n = face_tets(M, c->RF.a[i], c->RF.a[i + 1], c->RF.a[i + 2], tf);
        for (int j = 0; j < n; ++j)
            if (M->inR[tf[j] >> 2] != s) { c->status = ST_EXEMPT; c->reason = EX_RFTET; return; }
    }
    /* (d) boundary faces: faces of region tets that are not region subfaces
       and whose other side is the hull, a non-region tet, or a constraint;
       p must lie strictly on the inner side of each */
    for (int i = 0; i < c->RT.n; ++i) {
        int t = c->RT.a[i];
        const OTet* T = &M->T[t];
        for (int f = 0; f < 4; ++f) {
            if (face_is_rf(M, c, t, f)) continue;
            int a = T->v[FI[f][0]], b = T->v[FI[f][1]], d = T->v[FI[f][2]];
            int nb = neighbour(M, t, f);
            int bnd = nb < 0 || M->inR[nb >> 2] != s || get_sf(M, a, b, d);
            if (!bnd) continue;
            if (qmo_orient3d(X(M, a), X(M, b), X(M, d), p) <= 0) { c->status = ST_EXEMPT; c->reason = EX_FACE; return; }
            iv_push(&c->bface, (t << 2) | f);
        }
    }
    /* (e) 2D boundary edges of R_F: p strictly on the inner side, in the
       facet's projection (the edge split by a subsegment point excluded) */
    for (int i = 0; i < c->RF.n; i += 3) {
        const int* g = &c->RF.a[i];
        int F = get_sf(M, g[0], g[1], g[2])->v[0], ax = M->faxis[F];
        static const int EP[3][3] = {{0, 1, 2}, {0, 2, 1}, {1, 2, 0}};
        for (int j = 0; j < 3; ++j) {
            int x = g[EP[j][0]], y = g[EP[j][1]], z = g[EP[j][2]];
            if (c->cls == CLS_SS && x == c->tup[0] && y == c->tup[1]) continue;
            int h[3];
            int bnd = get_ss(M, x, y) != NULL;
            if (!bnd) bnd = !facet_neighbour(M, g, x, y, F, h) || !rf_has(&c->RF, h);
            if (!bnd) continue;
            int oz = qmo_orient2d(ax, X(M, x), X(M, y), X(M, z));
            int op = qmo_orient2d(ax, X(M, x), X(M, y), p);
            if (op == 0 || op != oz) { c->status = ST_EXEMPT; c->reason = EX_EDGE2D; return; }
            for (int q = 0; q < c->bedge.n; q += 4)      /* one new subface per edge */
                if (c->bedge.a[q] == x && c->bedge.a[q + 1] == y) { c->status = ST_EXEMPT; c->reason = EX_EDGE2D; return; }
            int tf[2];
            int one = face_tets(M, g[0], g[1], g[2], tf) == 1;
            iv_push(&c->bedge, x); iv_push(&c->bedge, y); iv_push(&c->bedge, F); iv_push(&c->bedge, one);
        }
    }
    /* (f) the boundary faces close up around p: every edge of a boundary
       face lies on exactly two boundary faces, or on exactly one when it is
       a 2D boundary edge of a region subface with a tet on one side only;
       every 2D boundary edge lies on as many boundary faces */
    for (int i = 0; i < c->bface.n; ++i) {
        int t = c->bface.a[i] >> 2, f = c->bface.a[i] & 3;
        const int* v = M->T[t].v;
        int fv[3] = {v[FI[f][0]], v[FI[f][1]], v[FI[f][2]]};
        for (int j = 0; j < 3; ++j) {
            int x = fv[j], y = fv[(j + 1) % 3];
            if (count_bfaces(M, c, x, y) != want_bfaces(c, x, y)) { c->status = ST_EXEMPT; c->reason = EX_MANIFOLD; return; }
        }
    }
    for (int q = 0; q < c->bedge.n; q += 4) {
        int x = c->bedge.a[q], y = c->bedge.a[q + 1];
        if (count_bfaces(M, c, x, y) != want_bfaces(c, x, y)) { c->status = ST_EXEMPT; c->reason = EX_MANIFOLD; return; }
    }
    /* (g) the mesh stays a CDT (Section 2: the triangulation is a CDT at the
       end of every round).  Each new interior face (x, y, p) that is not a
       new subface separates the new tets on the two boundary faces sharing
       edge xy; it must be locally Delaunay: the third vertex of the other
       boundary face is not strictly inside the circumsphere of the first
       new tet (x, y, z, p), which is positively oriented by (d).  With every
       other face of the new tets locally Delaunay by construction (an outer
       tet's sphere excludes p), this keeps every non-subface face of the
       mesh locally Delaunay, i.e. the mesh a CDT (constrained Delaunay
       lemma).  Without the check, a cavity that wraps more than half-way
       around a constraint edge can leave a face that is not. */
    for (int i = 0; i < c->bface.n; ++i) {
        const int* v = M->T[c->bface.a[i] >> 2].v;
        int f = c->bface.a[i] & 3;
        int fv[3] = {v[FI[f][0]], v[FI[f][1]], v[FI[f][2]]};
        for (int j = 0; j < 3; ++j) {
            int x = fv[j], y = fv[(j + 1) % 3];
            if (is_bedge(c, x, y)) continue;
            for (int i2 = i + 1; i2 < c->bface.n; ++i2) {
                const int* w = M->T[c->bface.a[i2] >> 2].v;
                int g = c->bface.a[i2] & 3;
                int hx = 0, hy = 0, apex = -1;
                for (int r = 0; r < 3; ++r) {
                    int u = w[FI[g][r]];
                    if (u == x) hx = 1; else if (u == y) hy = 1; else apex = u;
                }
                if (!hx || !hy) continue;
                if (qmo_insphere(X(M, fv[0]), X(M, fv[1]), X(M, fv[2]), p, X(M, apex)) > 0) {
                    c->status = ST_EXEMPT; c->reason = EX_DELAUNAY; return;
                }
            }
        }
    }
    /* claim set: region tets plus the tets across boundary faces */
    for (int i = 0; i < c->RT.n; ++i) iv_push(&c->claim, c->RT.a[i]);
    for (int i = 0; i < c->bface.n; ++i) {
        int nb = neighbour(M, c->bface.a[i] >> 2, c->bface.a[i] & 3);
        if (nb >= 0 && !iv_has(&c->claim, nb >> 2)) iv_push(&c->claim, nb >> 2);
    }
    c->status = ST_OK;
}

/* evaluate one candidate (steps 2-5) */
static void evaluate(Mesh* M, Cand* c) {
    int s = ++M->serial;
    split_point(M, c);
    for (int k = 0; k < 3; ++k)
        if (!isfinite(c->p[k])) { c->status = ST_EXEMPT; c->reason = EX_NONFINITE; return; }
    if (c->cls == CLS_SS) {
        int a = c->tup[0], b = c->tup[1];
        IV et = {0};
        edge_tets(M, a, b, &et);
        for (int i = 0; i < et.n; ++i) add_seed_tet(M, c, et.a[i], s);
        iv_free(&et);
        IV sfs = {0};
        edge_subfaces(M, a, b, &sfs);
        for (int q = 0; q < sfs.n; ++q) iv_push(&c->RF, sfs.a[q]);
        iv_free(&sfs);
        grow_rf(M, c);
    } else if (c->cls == CLS_SF) {
        int g[3];
        if (walk2d(M, c, c->tup, g)) return;
        iv_push(&c->RF, g[0]); iv_push(&c->RF, g[1]); iv_push(&c->RF, g[2]);
        grow_rf(M, c);
    } else {
        int t;
        if (walk3d(M, c, c->slot, &t)) return;
        add_seed_tet(M, c, t, s);
    }
    /* tets on region subfaces are seeds as well */
    for (int i = 0; i < c->RF.n; i += 3) {
        int tf[2], n = face_tets(M, c->RF.a[i], c->RF.a[i + 1], c->RF.a[i + 2], tf);
        for (int j = 0; j < n; ++j) add_seed_tet(M, c, tf[j] >> 2, s);
    }
    grow_rt(M, c, s);
    validate(M, c, s);
}

/* ---- Step 1: classify ---------------------------------------------- */
static int cmp_cand(const void* x, const void* y) {
    const Cand* a = (const Cand*)x; const Cand* b = (const Cand*)y;
    if (a->key != b->key) return a->key > b->key ? -1 : 1;   /* descending key */
    for (int i = 0; i < a->ntup; ++i)
        if (a->tup[i] != b->tup[i]) return a->tup[i] < b->tup[i] ? -1 : 1;
    return 0;
}

typedef struct { Cand* c; int n, cap; } CandList;
static Cand* cl_push(CandList* L) {
    if (L->n == L->cap) { L->cap = L->cap ? 2 * L->cap : 256; L->c = (Cand*)realloc(L->c, sizeof(Cand) * (size_t)L->cap); }
    Cand* c = &L->c[L->n++];
    memset(c, 0, sizeof *c);
    return c;
}

/* subsegment ab is encroached when queued or when a vertex of its link
   (an apex of a tet around ab) lies strictly inside its diametral ball */
static int ss_encroached(const Mesh* M, int a, int b, int flags) {
    if (flags & FL_QUEUED) return 1;
    IV et = {0};
    edge_tets(M, a, b, &et);
    int enc = 0;
    for (int i = 0; i < et.n && !enc; ++i)
        for (int k = 0; k < 4 && !enc; ++k) {
            int v = M->T[et.a[i]].v[k];
            if (v != a && v != b && qmo_segdot(X(M, a), X(M, b), X(M, v)) < 0) enc = 1;
        }
    iv_free(&et);
    return enc;
}

/* subface abc is encroached when queued or when the apex of one of its
   tets lies strictly inside its equatorial ball */
static int sf_encroached(const Mesh* M, const int* g, int flags) {
    if (flags & FL_QUEUED) return 1;
    int tf[2], n = face_tets(M, g[0], g[1], g[2], tf);
    for (int j = 0; j < n; ++j) {
        int apex = M->T[tf[j] >> 2].v[tf[j] & 3];
        if (qmo_facedot(X(M, g[0]), X(M, g[1]), X(M, g[2]), X(M, apex)) < 0) return 1;
    }
    return 0;
}

/* `only` = CLS_NONE: the round class is the first class with candidates
   (Section 2, "in this order"); otherwise that class alone is classified
   (the sub-phase reading, qmo_set_subphases). */
static int classify(Mesh* M, CandList* L, int only) {
    L->n = 0;
    if (only == CLS_NONE || only == CLS_SS)
    for (size_t i = 0; i < M->ss.cap; ++i) {
        HE* e = &M->ss.e[i];
        if (e->st != 1 || (e->v[1] & FL_EXEMPT)) continue;
        if (!ss_encroached(M, e->k[0], e->k[1], e->v[1])) continue;
        Cand* c = cl_push(L); c->cls = CLS_SS; c->ntup = 2; c->tup[0] = e->k[0]; c->tup[1] = e->k[1];
    }
    if (L->n) return CLS_SS;
    if (only == CLS_NONE || only == CLS_SF)
    for (size_t i = 0; i < M->sf.cap; ++i) {
        HE* e = &M->sf.e[i];
        if (e->st != 1 || (e->v[1] & FL_EXEMPT)) continue;
        if (!sf_encroached(M, e->k, e->v[1])) continue;
        Cand* c = cl_push(L); c->cls = CLS_SF; c->ntup = 3; memcpy(c->tup, e->k, 3 * sizeof(int));
    }
    if (L->n) return CLS_SF;
    if (only == CLS_NONE || only == CLS_TET)
    for (int t = 0; t < M->nt; ++t) {
        const OTet* T = &M->T[t];
        if (!T->alive || T->exempt) continue;
        int v[4]; memcpy(v, T->v, sizeof v); sort4(v);
        if (!qmo_is_bad(X(M, v[0]), X(M, v[1]), X(M, v[2]), X(M, v[3]), M->B2)) continue;
        Cand* c = cl_push(L); c->cls = CLS_TET; c->ntup = 4; memcpy(c->tup, v, sizeof v); c->slot = t;
    }
    if (L->n) return CLS_TET;
    return CLS_NONE;
}

/* ---- Step 7: insert ------------------------------------------------ */
static int insert_point(Mesh* M, Cand* c, int pid) {
    if (pid >= M->capv) {
        M->capv = 2 * M->capv + 16;
        M->V = (double(*)[3])realloc(M->V, sizeof(double) * 3 * (size_t)M->capv);
        M->vt = (int*)realloc(M->vt, sizeof(int) * (size_t)M->capv);
    }
    memcpy(M->V[pid], c->p, sizeof c->p);
    M->vt[pid] = -1;
    M->nv = pid + 1;
    /* new tets: p joined to every boundary face (read before deleting) */
    int nb = c->bface.n;
    int* nv4 = (int*)malloc(sizeof(int) * 4 * (size_t)(nb ? nb : 1));
    for (int i = 0; i < nb; ++i) {
        int t = c->bface.a[i] >> 2, f = c->bface.a[i] & 3;
        const int* v = M->T[t].v;
        nv4[4 * i] = v[FI[f][0]]; nv4[4 * i + 1] = v[FI[f][1]]; nv4[4 * i + 2] = v[FI[f][2]]; nv4[4 * i + 3] = pid;
    }
    for (int i = 0; i < c->RT.n; ++i) del_tet(M, c->RT.a[i]);
    for (int i = 0; i < c->RF.n; i += 3) {
        int k[4] = {c->RF.a[i], c->RF.a[i + 1], c->RF.a[i + 2], -1};
        HE* e = hm_get(&M->sf, k);
        if (e) hm_del(&M->sf, e);
    }
    for (int i = 0; i < nb; ++i) if (add_tet(M, &nv4[4 * i]) < 0) { free(nv4); return -1; }
    free(nv4);
    for (int i = 0; i < c->bedge.n; i += 4) {
        int k[4]; key3(k, c->bedge.a[i], c->bedge.a[i + 1], pid);
        HE* e = hm_put(&M->sf, k); e->v[0] = c->bedge.a[i + 2]; e->v[1] = 0;
    }
    if (c->cls == CLS_SS) {
        int k[4]; key2(k, c->tup[0], c->tup[1]);
        HE* e = hm_get(&M->ss, k);
        int seg = e->v[0];
        hm_del(&M->ss, e);
        key2(k, c->tup[0], pid); e = hm_put(&M->ss, k); e->v[0] = seg; e->v[1] = 0;
        key2(k, c->tup[1], pid); e = hm_put(&M->ss, k); e->v[0] = seg; e->v[1] = 0;
    }
    return 0;
}

/* ---------------------------------------------------------------- API */
#define QMO_NSTAT 17
/* per-round record: class, candidates, ok, rejected, exempt, kept,
   exempt by reason [1..9] in slots 6..14, vertices after, tets after */

#define QMO_NCHECK 9
int qmo_check(int nv, const double* xyz, int nt, const int* tets, int nsf, const int* sf,
              int nss, const int* ss, const int* ss_seg, double B, int* out, double* vol);

/* The sub-phase reading of Section 2's "in this order": every round takes
   the three classes in turn (subsegments, subfaces, bad tets), each as a
   round of its own with that class classified alone; a class without
   candidates is passed over without counting a round, and the refinement
   ends when the three classes in a row have none. */
static int g_subphases = 0;
void qmo_set_subphases(int on) { g_subphases = on; }

/* Resuming a refinement that the round guard stopped.  What the rounds
   carry beyond the mesh is a flag pair per subsegment and subface (queued by
   a rejected point, exempted by the filtering of Section 2), an exempt flag
   per bad tet whose point was filtered away, and h_min, fixed by the first
   input's shortest edge.  With a resume state set, qmo_refine takes these
   (aligned with its input arrays) instead of starting from clear flags, and
   the sub-phase reading starts at `next_class`. */
static const unsigned char *g_res_tfl = NULL, *g_res_sfl = NULL, *g_res_ssl = NULL;
static double g_res_hmin2 = 0.0;
static int g_res_on = 0, g_res_next = 0;
void qmo_set_resume(const unsigned char* tfl, const unsigned char* sfl, const unsigned char* ssl, double hmin2,
                    int next_class) {
    g_res_tfl = tfl; g_res_sfl = sfl; g_res_ssl = ssl; g_res_hmin2 = hmin2; g_res_next = next_class; g_res_on = 1;
}
void qmo_clear_resume(void) { g_res_on = 0; g_res_tfl = g_res_sfl = g_res_ssl = NULL; }

/* When set, every round ends with qmo_check on the current mesh, and its
   counts are kept per round (qmo_result_round_checks). */
static int g_round_check = 0;
void qmo_set_round_check(int on) { g_round_check = on; }

/* Test hook: record every candidate of round g_dump_round after the
   selection, for the brute-force pins of the region and the greedy set.
   Per candidate, ints: class, tuple length, tuple (4, -1 padded), key (high,
   low 32 bits), status, reason, kept, then the counts of region tets, region
   subfaces and claimed tets, then the region tets and claimed tets as sorted
   vertex-id quadruples and the region subfaces as sorted triples; doubles:
   the splitting point. */
static int g_dump_round = -1;
static IV g_dump_i;
static double* g_dump_d = NULL;
static int g_dump_nd = 0, g_dump_n = 0;
void qmo_set_dump_round(int r) {
    g_dump_round = r;
    iv_free(&g_dump_i);
    free(g_dump_d); g_dump_d = NULL; g_dump_nd = 0; g_dump_n = 0;
}
int qmo_dump_sizes(int* out) { out[0] = g_dump_i.n; out[1] = g_dump_nd; return g_dump_n; }
void qmo_dump_copy(int* ib, double* db) {
    if (g_dump_i.n) memcpy(ib, g_dump_i.a, sizeof(int) * (size_t)g_dump_i.n);
    if (g_dump_nd) memcpy(db, g_dump_d, sizeof(double) * (size_t)g_dump_nd);
}
static void dump_tet(const Mesh* M, int t) {
    int v[4]; memcpy(v, M->T[t].v, sizeof v); sort4(v);
    for (int k = 0; k < 4; ++k) iv_push(&g_dump_i, v[k]);
}
static void dump_round(const Mesh* M, const CandList* L) {
    g_dump_n = L->n;
    g_dump_d = (double*)malloc(sizeof(double) * 3 * (size_t)(L->n ? L->n : 1));
    g_dump_nd = 3 * L->n;
    for (int i = 0; i < L->n; ++i) {
        const Cand* c = &L->c[i];
        iv_push(&g_dump_i, c->cls); iv_push(&g_dump_i, c->ntup);
        for (int k = 0; k < 4; ++k) iv_push(&g_dump_i, k < c->ntup ? c->tup[k] : -1);
        iv_push(&g_dump_i, (int)(uint32_t)(c->key >> 32)); iv_push(&g_dump_i, (int)(uint32_t)c->key);
        iv_push(&g_dump_i, c->status); iv_push(&g_dump_i, c->reason); iv_push(&g_dump_i, c->kept);
        iv_push(&g_dump_i, c->RT.n); iv_push(&g_dump_i, c->RF.n / 3); iv_push(&g_dump_i, c->claim.n);
        for (int j = 0; j < c->RT.n; ++j) dump_tet(M, c->RT.a[j]);
        for (int j = 0; j < c->claim.n; ++j) dump_tet(M, c->claim.a[j]);
        for (int j = 0; j < c->RF.n; ++j) iv_push(&g_dump_i, c->RF.a[j]);
        memcpy(g_dump_d + 3 * i, c->p, sizeof c->p);
    }
}

typedef struct qmo_result {
    unsigned char *tfl, *sfl, *ssl;   /* state after the run, aligned with tets, sf, ss */
    double hmin2; int next_class;     /* h_min^2 used; sub-phase due next (sub-phase reading) */
    int* rcheck;                  /* QMO_NCHECK ints per round (round checks on) */
    int* lastc; int nlastc;       /* last round: 9 ints per candidate */
    int nv, nt, nsf, nss, rounds, status;
    double* xyz; int* tets; int* sf; int* sf_facet; int* ss; int* ss_seg;
    int* rstats; int nrstats;
    double seconds;
} qmo_result;

/* the current mesh as plain arrays, checked by qmo_check */
static void round_check(const Mesh* M, double B, int* out) {
    int nt = 0;
    for (int t = 0; t < M->nt; ++t) nt += M->T[t].alive;
    int* tets = (int*)malloc(sizeof(int) * 4 * (size_t)(nt + 1));
    for (int t = 0, j = 0; t < M->nt; ++t) if (M->T[t].alive) memcpy(&tets[4 * j++], M->T[t].v, 4 * sizeof(int));
    int nsf = (int)M->sf.n, nss = (int)M->ss.n;
    int* sf = (int*)malloc(sizeof(int) * 3 * (size_t)(nsf + 1));
    int* ss = (int*)malloc(sizeof(int) * 2 * (size_t)(nss + 1));
    int* sg = (int*)malloc(sizeof(int) * (size_t)(nss + 1));
    for (size_t i = 0, j = 0; i < M->sf.cap; ++i)
        if (M->sf.e[i].st == 1) { memcpy(&sf[3 * j], M->sf.e[i].k, 3 * sizeof(int)); j++; }
    for (size_t i = 0, j = 0; i < M->ss.cap; ++i)
        if (M->ss.e[i].st == 1) { memcpy(&ss[2 * j], M->ss.e[i].k, 2 * sizeof(int)); sg[j] = M->ss.e[i].v[0]; j++; }
    double vol;
    qmo_check(M->nv, &M->V[0][0], nt, tets, nsf, sf, nss, ss, sg, B, out, &vol);
    free(tets); free(sf); free(ss); free(sg);
}

static void apply_flags(Mesh* M, CandList* L) {
    for (int i = 0; i < L->n; ++i) {
        Cand* c = &L->c[i];
        if (c->status == ST_REJECT) {
            for (int q = 0; q < c->Q.n; q += 4) {
                int k[4] = {c->Q.a[q + 1], c->Q.a[q + 2], c->Q.a[q + 3], -1};
                HE* e = c->Q.a[q] == 0 ? hm_get(&M->ss, k) : hm_get(&M->sf, k);
                if (e) e->v[1] |= FL_QUEUED;
            }
        } else if (c->status == ST_EXEMPT) {
            if (c->cls == CLS_SS) { HE* e = get_ss(M, c->tup[0], c->tup[1]); if (e) e->v[1] |= FL_EXEMPT; }
            else if (c->cls == CLS_SF) { HE* e = get_sf(M, c->tup[0], c->tup[1], c->tup[2]); if (e) e->v[1] |= FL_EXEMPT; }
            else M->T[c->slot].exempt = 1;
        }
    }
}

/*
 * qmo_refine: run the refinement.
 *   xyz[nv*3]                 vertex coordinates (lattice multiples of 2^-53)
 *   tets[nt*4]                positively oriented tets of the input CDT
 *   sf[nsf*3], sf_facet[nsf]  subfaces and their facet ids
 *   ss[nss*2], ss_seg[nss]    subsegments and their segment ids
 *   ftri[nftri*3], ftri_facet PLC polygons as triangles (facet projection axis
 *                             is taken from the first triangle of each facet)
 *   B                         radius-edge bound
 *   hmin_factor               h_min = hmin_factor * shortest input edge
 *   max_rounds                round guard (status 1 when reached)
 *   max_kept                  if > 0, insert at most this many points per round
 * Returns 0 and a result, or a negative code for invalid input.
 */
int qmo_refine(int nv, const double* xyz, int nt, const int* tets,
               int nsf, const int* sf, const int* sf_facet,
               int nss, const int* ss, const int* ss_seg,
               int nftri, const int* ftri, const int* ftri_facet,
               double B, double hmin_factor, int max_rounds, int max_kept,
               qmo_result** out) {
    struct timespec t0, t1;
    Mesh Mo; Mesh* M = &Mo;
    memset(M, 0, sizeof *M);
    M->capv = nv + 16;
    M->V = (double(*)[3])malloc(sizeof(double) * 3 * (size_t)M->capv);
    M->vt = (int*)malloc(sizeof(int) * (size_t)M->capv);
    memcpy(M->V, xyz, sizeof(double) * 3 * (size_t)nv);
    for (int i = 0; i < nv; ++i) M->vt[i] = -1;
    M->nv = nv;
    hm_init(&M->faces, (size_t)nt * 6);
    hm_init(&M->sf, (size_t)nsf * 4 + 64);
    hm_init(&M->ss, (size_t)nss * 4 + 64);
    double l2 = INFINITY;
    for (int t = 0; t < nt; ++t) {
        const int* v = &tets[4 * t];
        for (int k = 0; k < 4; ++k) if (v[k] < 0 || v[k] >= nv) return -1;
        if (qmo_orient3d(X(M, v[0]), X(M, v[1]), X(M, v[2]), X(M, v[3])) <= 0) return -2;
        int ti = add_tet(M, v);
        if (ti < 0) return -3;
        if (g_res_on && g_res_tfl) M->T[ti].exempt = g_res_tfl[t] & 1;
        for (int e = 0; e < 6; ++e) { double d = qmo_d2(X(M, v[EDGE[e][0]]), X(M, v[EDGE[e][1]])); if (d < l2) l2 = d; }
    }
    for (int i = 0; i < nsf; ++i) {
        int k[4]; key3(k, sf[3 * i], sf[3 * i + 1], sf[3 * i + 2]);
        if (!hm_get(&M->faces, k)) return -4;
        HE* e = hm_put(&M->sf, k); e->v[0] = sf_facet[i]; e->v[1] = g_res_on && g_res_sfl ? (g_res_sfl[i] & 3) : 0;
    }
    for (int i = 0; i < nss; ++i) {
        int k[4]; key2(k, ss[2 * i], ss[2 * i + 1]);
        IV et = {0}; edge_tets(M, k[0], k[1], &et);
        int n = et.n; iv_free(&et);
        if (!n) return -5;
        HE* e = hm_put(&M->ss, k); e->v[0] = ss_seg[i]; e->v[1] = g_res_on && g_res_ssl ? (g_res_ssl[i] & 3) : 0;
    }
    int nfacet = 0;
    for (int i = 0; i < nftri; ++i) if (ftri_facet[i] + 1 > nfacet) nfacet = ftri_facet[i] + 1;
    M->faxis = (int*)malloc(sizeof(int) * (size_t)(nfacet + 1));
    for (int f = 0; f < nfacet; ++f) M->faxis[f] = -1;
    for (int i = 0; i < nftri; ++i) {
        int F = ftri_facet[i];
        if (M->faxis[F] >= 0) continue;
        const double *a = X(M, ftri[3 * i]), *b = X(M, ftri[3 * i + 1]), *d = X(M, ftri[3 * i + 2]);
        double u[3], w[3];
        for (int k = 0; k < 3; ++k) { u[k] = b[k] - a[k]; w[k] = d[k] - a[k]; }
        double n[3] = {fabs(u[1] * w[2] - u[2] * w[1]), fabs(u[2] * w[0] - u[0] * w[2]), fabs(u[0] * w[1] - u[1] * w[0])};
        int ax = 0;
        if (n[1] > n[ax]) ax = 1;
        if (n[2] > n[ax]) ax = 2;
        M->faxis[F] = ax;
    }
    M->nfacet = nfacet;
    M->B2 = B * B;
    M->hmin2 = g_res_on ? g_res_hmin2 : (hmin_factor * hmin_factor) * l2;

    qmo_result* R = (qmo_result*)calloc(1, sizeof *R);
    int rcap = 256;
    R->rstats = (int*)calloc((size_t)rcap * QMO_NSTAT, sizeof(int));
    if (g_round_check) R->rcheck = (int*)calloc((size_t)rcap * QMO_NCHECK, sizeof(int));
    CandList L = {0};
    clock_gettime(CLOCK_MONOTONIC, &t0);
    int round = 0;
    R->status = 0;
    int sub = g_res_on ? g_res_next : CLS_SS, empty_turns = 0;
    for (;;) {
        if (round >= max_rounds) { R->status = 1; break; }
        int cls = classify(M, &L, g_subphases ? sub : CLS_NONE);
        if (g_subphases) {
            sub = (sub + 1) % 3;
            if (cls == CLS_NONE) {
                if (++empty_turns == 3) break;
                continue;
            }
            empty_turns = 0;
        }
        if (cls == CLS_NONE) break;
        for (int i = 0; i < L.n; ++i) {
            Cand* c = &L.c[i];
            c->key = cand_key(c);
        }
        qsort(L.c, (size_t)L.n, sizeof(Cand), cmp_cand);
        int nok = 0, nrej = 0, nex = 0, byr[EX_NREASON] = {0};
        for (int i = 0; i < L.n; ++i) {
            Cand* c = &L.c[i];
            evaluate(M, c);
            c->kept = 0;
            if (c->status == ST_OK) nok++;
            else if (c->status == ST_REJECT) nrej++;
            else { nex++; byr[c->reason]++; }
        }
        /* Step 6: greedy maximal set of disjoint claim sets, by priority */
        int nkept = 0;
        for (int i = 0; i < L.n; ++i) {
            Cand* c = &L.c[i];
            if (c->status != ST_OK) continue;
            if (max_kept > 0 && nkept >= max_kept) break;
            int free_ = 1;
            for (int j = 0; j < c->claim.n && free_; ++j) if (M->claimed[c->claim.a[j]] == round) free_ = 0;
            if (!free_) continue;
            for (int j = 0; j < c->claim.n; ++j) M->claimed[c->claim.a[j]] = round;
            c->kept = 1; nkept++;
        }
        if (round == g_dump_round) dump_round(M, &L);
        apply_flags(M, &L);
        int pid = M->nv;
        for (int i = 0; i < L.n; ++i) {
            Cand* c = &L.c[i];
            if (!c->kept) continue;
            if (insert_point(M, c, pid++) < 0) { R->status = -7; goto finish; }
        }
        if (round >= rcap) {
            R->rstats = (int*)realloc(R->rstats, sizeof(int) * QMO_NSTAT * (size_t)rcap * 2);
            memset(R->rstats + QMO_NSTAT * rcap, 0, sizeof(int) * QMO_NSTAT * (size_t)rcap);
            if (R->rcheck) {
                R->rcheck = (int*)realloc(R->rcheck, sizeof(int) * QMO_NCHECK * (size_t)rcap * 2);
                memset(R->rcheck + QMO_NCHECK * rcap, 0, sizeof(int) * QMO_NCHECK * (size_t)rcap);
            }
            rcap *= 2;
        }
        int* rs = R->rstats + QMO_NSTAT * round;
        rs[0] = cls; rs[1] = L.n; rs[2] = nok; rs[3] = nrej; rs[4] = nex; rs[5] = nkept;
        for (int r = 1; r < EX_NREASON; ++r) rs[5 + r] = byr[r];
        rs[15] = M->nv;
        int live = 0; for (int t = 0; t < M->nt; ++t) live += M->T[t].alive;
        rs[16] = live;
        if (R->rcheck) round_check(M, B, R->rcheck + QMO_NCHECK * round);
        free(R->lastc);
        R->lastc = (int*)malloc(sizeof(int) * 9 * (size_t)(L.n ? L.n : 1));
        R->nlastc = L.n;
        for (int i = 0; i < L.n; ++i) {
            Cand* c = &L.c[i];
            int* o = R->lastc + 9 * i;
            for (int k = 0; k < 4; ++k) o[k] = k < c->ntup ? c->tup[k] : -1;
            o[4] = c->status; o[5] = c->status == ST_EXEMPT ? c->reason : 0; o[6] = c->kept;
            o[7] = c->status == ST_OK ? c->RT.n : 0; o[8] = c->status == ST_OK ? c->bface.n : 0;
        }
        for (int i = 0; i < L.n; ++i) cand_free(&L.c[i]);
        L.n = 0;
        round++;
    }
finish:
    clock_gettime(CLOCK_MONOTONIC, &t1);
    for (int i = 0; i < L.n; ++i) cand_free(&L.c[i]);
    free(L.c);
    R->seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    R->rounds = round;
    R->nrstats = round;
    R->nv = M->nv;
    R->xyz = (double*)malloc(sizeof(double) * 3 * (size_t)M->nv);
    memcpy(R->xyz, M->V, sizeof(double) * 3 * (size_t)M->nv);
    int live = 0; for (int t = 0; t < M->nt; ++t) live += M->T[t].alive;
    R->nt = live;
    R->tets = (int*)malloc(sizeof(int) * 4 * (size_t)(live ? live : 1));
    R->tfl = (unsigned char*)malloc((size_t)(live ? live : 1));
    for (int t = 0, j = 0; t < M->nt; ++t)
        if (M->T[t].alive) { R->tfl[j] = M->T[t].exempt; memcpy(&R->tets[4 * j++], M->T[t].v, 4 * sizeof(int)); }
    R->nsf = (int)M->sf.n;
    R->sf = (int*)malloc(sizeof(int) * 3 * (size_t)(R->nsf + 1));
    R->sf_facet = (int*)malloc(sizeof(int) * (size_t)(R->nsf + 1));
    R->sfl = (unsigned char*)malloc((size_t)(R->nsf + 1));
    for (size_t i = 0, j = 0; i < M->sf.cap; ++i)
        if (M->sf.e[i].st == 1) {
            memcpy(&R->sf[3 * j], M->sf.e[i].k, 3 * sizeof(int)); R->sf_facet[j] = M->sf.e[i].v[0];
            R->sfl[j] = (unsigned char)(M->sf.e[i].v[1] & 3); j++;
        }
    R->nss = (int)M->ss.n;
    R->ss = (int*)malloc(sizeof(int) * 2 * (size_t)(R->nss + 1));
    R->ss_seg = (int*)malloc(sizeof(int) * (size_t)(R->nss + 1));
    R->ssl = (unsigned char*)malloc((size_t)(R->nss + 1));
    for (size_t i = 0, j = 0; i < M->ss.cap; ++i)
        if (M->ss.e[i].st == 1) {
            memcpy(&R->ss[2 * j], M->ss.e[i].k, 2 * sizeof(int)); R->ss_seg[j] = M->ss.e[i].v[0];
            R->ssl[j] = (unsigned char)(M->ss.e[i].v[1] & 3); j++;
        }
    R->hmin2 = M->hmin2;
    R->next_class = g_subphases ? sub : 0;
    hm_free(&M->faces); hm_free(&M->sf); hm_free(&M->ss);
    free(M->V); free(M->vt); free(M->T); free(M->inR); free(M->tested); free(M->claimed); free(M->instar); free(M->faxis);
    *out = R;
    return 0;
}

void qmo_result_counts(const qmo_result* R, int* out) {
    out[0] = R->nv; out[1] = R->nt; out[2] = R->nsf; out[3] = R->nss; out[4] = R->rounds; out[5] = R->status;
}
double qmo_result_seconds(const qmo_result* R) { return R->seconds; }
void qmo_result_copy(const qmo_result* R, double* xyz, int* tets, int* sf, int* sf_facet, int* ss, int* ss_seg, int* rstats) {
    memcpy(xyz, R->xyz, sizeof(double) * 3 * (size_t)R->nv);
    memcpy(tets, R->tets, sizeof(int) * 4 * (size_t)R->nt);
    memcpy(sf, R->sf, sizeof(int) * 3 * (size_t)R->nsf);
    memcpy(sf_facet, R->sf_facet, sizeof(int) * (size_t)R->nsf);
    memcpy(ss, R->ss, sizeof(int) * 2 * (size_t)R->nss);
    memcpy(ss_seg, R->ss_seg, sizeof(int) * (size_t)R->nss);
    memcpy(rstats, R->rstats, sizeof(int) * QMO_NSTAT * (size_t)R->nrstats);
}
int qmo_result_round_checks(const qmo_result* R, int* buf) {
    if (!R->rcheck) return 0;
    if (buf) memcpy(buf, R->rcheck, sizeof(int) * QMO_NCHECK * (size_t)R->nrstats);
    return R->nrstats;
}
/* the state after the run, aligned with the arrays of qmo_result_copy;
   returns the sub-phase due next */
int qmo_result_state(const qmo_result* R, unsigned char* tfl, unsigned char* sfl, unsigned char* ssl, double* hmin2) {
    memcpy(tfl, R->tfl, (size_t)R->nt);
    memcpy(sfl, R->sfl, (size_t)R->nsf);
    memcpy(ssl, R->ssl, (size_t)R->nss);
    *hmin2 = R->hmin2;
    return R->next_class;
}
int qmo_result_lastc(const qmo_result* R, int* buf) {
    if (buf) memcpy(buf, R->lastc, sizeof(int) * 9 * (size_t)R->nlastc);
    return R->nlastc;
}
void qmo_result_free(qmo_result* R) {
    if (!R) return;
    free(R->lastc); free(R->rcheck); free(R->tfl); free(R->sfl); free(R->ssl);
    free(R->xyz); free(R->tets); free(R->sf); free(R->sf_facet); free(R->ss); free(R->ss_seg); free(R->rstats);
    free(R);
}

/* --- the library's call layout ---------------------------------------- */
/* qm_oracle_refine takes its arguments in the layout of the GPU library's
   refine call: a PLC, a mesh and options, each a struct with the same field
   order and types, and it answers with the library's return codes.  A test
   can then marshal one set of arguments and hand it to either engine.  The
   structs are declared here again (a call layout is an interface, not shared
   code).  Of the option flags, the sub-phase reading (1024) and forced equal
   priorities (128) change the run; early-stop blasting (256, timing-decided)
   and device arrays (1) are refused; the others only concern the GPU
   (profiling, device output, tier tests) and are ignored. */
typedef struct {
    int32_t nv; int32_t nseg; const int32_t* seg;
    int32_t nftri; const int32_t* ftri; const int32_t* ftri_facet;
} qmo_call_plc;
typedef struct {
    int32_t nv; const double* xyz; int32_t nt; const int32_t* tet;
    int32_t nsf; const int32_t* sf; const int32_t* sf_facet;
    int32_t nss; const int32_t* ss; const int32_t* ss_seg;
} qmo_call_mesh;
typedef struct { double B; double hmin_factor; int32_t max_rounds; int32_t max_kept; uint32_t flags; } qmo_call_options;

enum { QMO_CALL_INPUT_DEVICE = 1u, QMO_CALL_KEY_COLLIDE = 128u, QMO_CALL_EARLY_STOP = 256u,
       QMO_CALL_SUBPHASES = 1024u };

int qm_oracle_refine(const qmo_call_plc* plc, const qmo_call_mesh* in, const qmo_call_options* opt,
                     qmo_result** out) {
    if (!plc || !in || !opt || !out) return -1;                       /* invalid argument */
    if (opt->flags & (QMO_CALL_INPUT_DEVICE | QMO_CALL_EARLY_STOP)) return -1;
    if (!(opt->B > 0.0) || !(opt->hmin_factor >= 0.0) || opt->max_rounds < 0) return -1;
    if (in->nv < 8 || in->nt < 1 || in->nsf < 0 || in->nss < 0 || plc->nftri < 0) return -1;
    for (int i = 0; i < 3 * in->nv; ++i) {        /* coordinates in the cube, on the 2^-53 lattice */
        const double c = in->xyz[i], s = ldexp(c, 53);
        if (!(c >= 0.0 && c <= 1.0) || rint(s) != s) return -1;
    }
    const int sub0 = g_subphases;
    const uint64_t mask0 = g_key_mask;
    g_subphases = (opt->flags & QMO_CALL_SUBPHASES) != 0;
    if (opt->flags & QMO_CALL_KEY_COLLIDE) g_key_mask = 0xE000000000000000ull;
    int rc = qmo_refine(in->nv, in->xyz, in->nt, in->tet, in->nsf, in->sf, in->sf_facet, in->nss, in->ss,
                        in->ss_seg, plc->nftri, plc->ftri, plc->ftri_facet, opt->B, opt->hmin_factor,
                        opt->max_rounds, opt->max_kept, out);
    g_subphases = sub0;
    g_key_mask = mask0;
    if (rc == -1) return -1;                  /* ids out of range */
    if (rc < 0) return -2;                    /* not a conforming tetrahedralisation of the PLC */
    if ((*out)->status < 0) return -6;        /* an insertion failed: impossible state */
    return (*out)->status == 1 ? -4 : 0;      /* round guard reached: the result is still returned */
}

/* --- predicate entry points for the oracle's own pin tests ------------- */
int qmo_p_orient3d(const double* a, const double* b, const double* c, const double* d) { return qmo_orient3d(a, b, c, d); }
int qmo_p_insphere(const double* a, const double* b, const double* c, const double* d, const double* e) { return qmo_insphere(a, b, c, d, e); }
int qmo_p_orient2d(int ax, const double* a, const double* b, const double* c) { return qmo_orient2d(ax, a, b, c); }
int qmo_p_segdot(const double* a, const double* b, const double* v) { return qmo_segdot(a, b, v); }
int qmo_p_facedot(const double* a, const double* b, const double* c, const double* v) { return qmo_facedot(a, b, c, v); }
void qmo_c_midpoint(const double* a, const double* b, double* p) { qmo_midpoint(a, b, p); }
void qmo_c_tri_cc(const double* a, const double* b, const double* c, double* p) { qmo_tri_cc(a, b, c, p); }
void qmo_c_tet_cc(const double* a, const double* b, const double* c, const double* d, double* p, double* R2) { qmo_tet_cc(a, b, c, d, p, R2); }
int qmo_c_is_bad(const double* a, const double* b, const double* c, const double* d, double B) { return qmo_is_bad(a, b, c, d, B * B); }
uint64_t qmo_c_key(int cls, const int* ids, int n) { return qmo_key(cls, ids, n); }

/* ------------------------------------------------------------------------
 * Property checks on a mesh (used by the tests on oracle and GPU outputs).
 * out[0]  tets not positively oriented
 * out[1]  faces shared by more than two tets
 * out[2]  hull faces that are not subfaces
 * out[3]  interior non-subface faces that are not locally Delaunay
 *         (the apex across the face strictly inside the circumsphere)
 * out[4]  subfaces that are not faces of the mesh
 * out[5]  subsegments that are not edges of the mesh
 * out[6]  V - E + F - T (1 for a triangulated ball)
 * out[7]  bad tets (radius-edge ratio > B)
 * out[8]  subsegment chains broken (per segment: endpoint degree test)
 * vol[0]  total volume (FP64 sum of det/6)
 * By the constrained Delaunay lemma, out[3] == 0 (with every subface a face
 * of the mesh) means the mesh is a CDT of its subfaces and subsegments.
 * ---------------------------------------------------------------------- */
int qmo_check(int nv, const double* xyz, int nt, const int* tets, int nsf, const int* sf,
              int nss, const int* ss, const int* ss_seg, double B, int* out, double* vol) {
    memset(out, 0, sizeof(int) * 9);
    HMap fm, sfm, em;
    hm_init(&fm, (size_t)nt * 6); hm_init(&sfm, (size_t)nsf * 4 + 64); hm_init(&em, (size_t)nt * 8);
    const double (*V)[3] = (const double(*)[3])xyz;
    double vsum = 0;
    for (int i = 0; i < nsf; ++i) { int k[4]; key3(k, sf[3 * i], sf[3 * i + 1], sf[3 * i + 2]); hm_put(&sfm, k)->v[0] = 1; }
    for (int t = 0; t < nt; ++t) {
        const int* v = &tets[4 * t];
        if (qmo_orient3d(V[v[0]], V[v[1]], V[v[2]], V[v[3]]) <= 0) out[0]++;
        double u[3], w[3], z[3];
        for (int k = 0; k < 3; ++k) { u[k] = V[v[1]][k] - V[v[0]][k]; w[k] = V[v[2]][k] - V[v[0]][k]; z[k] = V[v[3]][k] - V[v[0]][k]; }
        vsum += (u[0] * (w[1] * z[2] - w[2] * z[1]) + u[1] * (w[2] * z[0] - w[0] * z[2]) + u[2] * (w[0] * z[1] - w[1] * z[0])) / 6.0;
        for (int f = 0; f < 4; ++f) {
            int k[4]; key3(k, v[FI[f][0]], v[FI[f][1]], v[FI[f][2]]);
            HE* e = hm_put(&fm, k);
            if (e->v[0] < 0) e->v[0] = (t << 2) | f; else if (e->v[1] < 0) e->v[1] = (t << 2) | f; else out[1]++;
        }
        for (int e = 0; e < 6; ++e) { int k[4]; key2(k, v[EDGE[e][0]], v[EDGE[e][1]]); hm_put(&em, k); }
        int s[4]; memcpy(s, v, sizeof s); sort4(s);
        if (qmo_is_bad(V[s[0]], V[s[1]], V[s[2]], V[s[3]], B * B)) out[7]++;
    }
    for (size_t i = 0; i < fm.cap; ++i) {
        HE* e = &fm.e[i];
        if (e->st != 1) continue;
        int issf = hm_get(&sfm, e->k) != NULL;
        if (e->v[1] < 0) { if (!issf) out[2]++; continue; }
        if (issf) continue;
        for (int side = 0; side < 2; ++side) {
            int t = e->v[side] >> 2, o = e->v[1 - side] >> 2, of = e->v[1 - side] & 3;
            const int* v = &tets[4 * t];
            int apex = tets[4 * o + of];
            if (qmo_insphere(V[v[0]], V[v[1]], V[v[2]], V[v[3]], V[apex]) > 0) { out[3]++; break; }
        }
    }
    for (int i = 0; i < nsf; ++i) { int k[4]; key3(k, sf[3 * i], sf[3 * i + 1], sf[3 * i + 2]); if (!hm_get(&fm, k)) out[4]++; }
    for (int i = 0; i < nss; ++i) { int k[4]; key2(k, ss[2 * i], ss[2 * i + 1]); if (!hm_get(&em, k)) out[5]++; }
    /* Euler characteristic over used vertices */
    char* used = (char*)calloc((size_t)nv, 1);
    int nvu = 0;
    for (int t = 0; t < 4 * nt; ++t) if (!used[tets[t]]) { used[tets[t]] = 1; nvu++; }
    out[6] = nvu - (int)em.n + (int)fm.n - nt;
    /* subsegment chains: per segment, each vertex has degree 2 except the two ends */
    HMap deg; hm_init(&deg, (size_t)nss * 4 + 64);
    for (int i = 0; i < nss; ++i)
        for (int j = 0; j < 2; ++j) { int k[4] = {ss_seg[i], ss[2 * i + j], -1, -1}; HE* e = hm_put(&deg, k); e->v[0] = e->v[0] < 0 ? 1 : e->v[0] + 1; }
    HMap ends; hm_init(&ends, 1024);
    for (size_t i = 0; i < deg.cap; ++i) {
        HE* e = &deg.e[i];
        if (e->st != 1) continue;
        if (e->v[0] > 2) out[8]++;
        if (e->v[0] == 1) { int k[4] = {e->k[0], -1, -1, -1}; HE* q = hm_put(&ends, k); q->v[0] = q->v[0] < 0 ? 1 : q->v[0] + 1; }
    }
    for (size_t i = 0; i < ends.cap; ++i) if (ends.e[i].st == 1 && ends.e[i].v[0] != 2) out[8]++;
    free(used); hm_free(&fm); hm_free(&sfm); hm_free(&em); hm_free(&deg); hm_free(&ends);
    *vol = vsum;
    return 0;
}

/* Brute-force global test: number of tets whose circumsphere strictly
   encloses some vertex of the mesh (0 for a Delaunay tetrahedralisation). */
int qmo_check_global(int nv, const double* xyz, int nt, const int* tets) {
    const double (*V)[3] = (const double(*)[3])xyz;
    char* used = (char*)calloc((size_t)nv, 1);
    for (int i = 0; i < 4 * nt; ++i) used[tets[i]] = 1;
    int bad = 0;
    for (int t = 0; t < nt; ++t) {
        const int* v = &tets[4 * t];
        for (int q = 0; q < nv; ++q) {
            if (!used[q] || q == v[0] || q == v[1] || q == v[2] || q == v[3]) continue;
            if (qmo_insphere(V[v[0]], V[v[1]], V[v[2]], V[v[3]], V[q]) > 0) { bad++; break; }
        }
    }
    free(used);
    return bad;
}
