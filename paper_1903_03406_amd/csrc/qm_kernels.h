// qm_kernels.h -- device kernels of one refinement round (gfx950).
//
// Round (paper, Section 2): classify elements in the order subsegments,
// subfaces, tetrahedra; compute splitting points; locate and grow each
// point's Delaunay region; filter; keep a maximal set of points whose regions
// are disjoint (priority marking); insert the kept points concurrently.
//
// Data layout in HBM (structure of arrays, slot-indexed):
//   X   double4[nv]     vertex coordinates (w unused)
//   TV  int[4*nt]       tet vertices, positively oriented; face f is opposite
//                       vertex f
//   TA  int[4*nt]       neighbour across face f as (t'<<2|f'), -1 on the hull
//   TF  int[4*nt]       facet id when face f is a subface, else -1 (both tets
//                       of an interior subface carry it)
//   TS  int[6*nt]       subsegment slot of each tet edge, else -1
//   TI  uint[nt]        bit0 alive, bit1 exempt, bits 4+f face queued,
//                       bits 8+f face exempt, bits 12-13 grow-tier hint,
//                       bits 14-31 cached classification (see TI_BADK)
//   SV  int2[nss]       subsegment endpoints (ascending); SSEG segment id;
//   SFL uint[nss]       bit0 queued, bit1 exempt, bits 2-3 cached link test;
//                       STET a tet holding the edge
// Every decision is a function of vertex ids and coordinates only; slots and
// launch order never change a result.
#pragma once
#include "qm_geom.h"

namespace qm {

enum { CLS_SS = 0, CLS_SF = 1, CLS_TET = 2, CLS_NONE = 3 };
enum { ST_OK = 0, ST_REJECT = 1, ST_EXEMPT = 2, ST_PENDING = 3, ST_OVERFLOW = 4, ST_POOLFULL = 5,
       ST_TOOBIG = 6, ST_OVERFLOW2 = 7, ST_LOST = 8 };   // LOST: stopped early (early-stop mode)
enum { EX_NONE = 0, EX_NONFINITE = 1, EX_WALK = 2, EX_ENC_EXEMPT = 3, EX_HMIN = 4,
       EX_RFTET = 5, EX_FACE = 6, EX_EDGE2D = 7, EX_MANIFOLD = 8, EX_DELAUNAY = 9,
       EX_NREASON = 10 };
enum { TI_ALIVE = 1u, TI_EXEMPT = 2u };
constexpr int TI_HINT_SHIFT = 12;   // bits 12-13: grow tier a bad tet's region needed (1 medium, 3 global)
// Cached classification (each is a function of the tet's own vertices, or of
// a subface's two apexes, so it holds until k_insert rewrites the tet or the
// neighbour across the face):
constexpr unsigned TI_BADK = 1u << 14;   // bad-tet test done
constexpr unsigned TI_BAD = 1u << 15;    // ... and the tet is bad
QMD unsigned ti_fknown(int f) { return 1u << (16 + f); }   // subface f: status below is current
QMD unsigned ti_fenc(int f) { return 1u << (20 + f); }     // subface f encroached by an apex
QMD unsigned ti_fcanon(int f) { return 1u << (24 + f); }   // this tet holds the canonical copy
QMD unsigned ti_fsub(int f) { return 1u << (28 + f); }     // face f is a subface (TF >= 0)
enum { SS_QUEUED = 1u, SS_EXEMPT = 2u, SS_KNOWN = 4u, SS_ENC = 8u };   // KNOWN/ENC: cached link test
constexpr int WALK_CAP = 1000000;
constexpr int RING_CAP = 4096;

struct Mesh {
    double4* X;
    int* TV; int* TA; int* TF; int* TS; unsigned* TI;
    int2* SV; int* SSEG; unsigned* SFL; int* STET;
    const int* FAX;
    int* err;             // this call's error word (broken preconditions, never expected)
    int nv, nt, nss;
    double B2, hmin2;
};

// candidates of one round, in priority order after sorting
struct Cands {
    int n;
    int* elem;            // SS: subsegment slot; SF: t<<2|f; TET: t
    unsigned long long* key;
    int4* tup;            // sorted vertex ids, padded with -1
    double4* p;           // splitting point (lattice)
    int* st;              // status after split/locate (ST_PENDING: go on)
    int* reason;
    int* seed;            // located tet (TET) or subface t<<2|f (SF)
    int2* qw;             // walk rejection target: (kind, handle)
    // region evaluation
    int* gst; int* greason;
    int* reg_off; int* reg_n;
    int* bf_off; int* bf_n;
    int* be_off; int* be_n;
    int* cl_off; int* cl_n;
    int* q_off; int* q_n;
    int* state;           // selection: 0 undecided, 1 kept, 2 dropped, 3 not a candidate
};

struct Pools {
    int4* be; int* cl; int* clc; int2* q;
    int cap_be, cap_cl, cap_q;
    int* ctr;             // [1] face records, [2] be, [3] cl, [4] q, [5] pool overflow
    // early-stop blasting (a non-parity mode): per-tet priority marks of this
    // grow pass, or null
    unsigned long long* es_mark;
    unsigned es_pass;
};

__constant__ int c_FI[4][3] = {{1, 3, 2}, {0, 2, 3}, {0, 3, 1}, {0, 1, 2}};
__constant__ int c_EV[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
__constant__ int c_EIDX[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};

QMD int4 ld4(const int* a, int t) { return *reinterpret_cast<const int4*>(a + 4 * (size_t)t); }
QMD int at4(int4 v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w)); }
QMD void xyz(const Mesh& M, int v, double* o) {
    double4 q = M.X[v];
    o[0] = q.x; o[1] = q.y; o[2] = q.z;
}
QMD int local_of(int4 v, int id) { return v.x == id ? 0 : (v.y == id ? 1 : (v.z == id ? 2 : (v.w == id ? 3 : -1))); }
QMD void sort3(int& a, int& b, int& c) {
    int t;
    if (b < a) { t = a; a = b; b = t; }
    if (c < b) { t = b; b = c; c = t; }
    if (b < a) { t = a; a = b; b = t; }
}
// canonical key of the subface on face f of t (same for both tets)
QMD int face_ckey(const Mesh& M, int t, int f) {
    int me = (t << 2) | f;
    int nb = M.TA[4 * (size_t)t + f];
    return (nb >= 0 && nb < me) ? nb : me;
}
QMD int edge_ss(const Mesh& M, int t, int4 v, int x, int y) {
    int lx = local_of(v, x), ly = local_of(v, y);
    return M.TS[6 * (size_t)t + c_EIDX[lx][ly]];
}

// Visit the tets around edge (a,b), starting at t0 which holds it.
// visit(t, u, w): u, w are the tet's vertices other than a and b.  A visit
// returning true stops the walk.  Returns false if the ring was cut short.
template <class F>
__device__ bool ring(const Mesh& M, int t0, int a, int b, F&& visit) {
    if (t0 < 0 || t0 >= M.nt) { atomicOr(M.err, 16); return false; }
    int4 v0 = ld4(M.TV, t0);
    int o[2], k = 0;
    for (int i = 0; i < 4; ++i) { int x = at4(v0, i); if (x != a && x != b && k < 2) o[k++] = x; }
    if (k != 2) { atomicOr(M.err, 16); return false; }   // t0 does not hold the edge
    if (visit(t0, o[0], o[1])) return true;
    bool closed = false;
    for (int dir = 0; dir < 2 && !closed; ++dir) {
        int t = t0, u = dir == 0 ? o[0] : o[1], w = dir == 0 ? o[1] : o[0];
        for (int step = 0; step < RING_CAP; ++step) {
            int4 vt = ld4(M.TV, t);
            int lu = local_of(vt, u);
            if (lu < 0) { atomicOr(M.err, 32); return false; }
            int nb = M.TA[4 * (size_t)t + lu];
            if (nb < 0) break;                       // hull: go the other way
            int tn = nb >> 2;
            if (tn >= M.nt) { atomicOr(M.err, 64); return false; }
            if (tn == t0) { closed = true; break; }
            int apex = M.TV[4 * (size_t)tn + (nb & 3)];
            if (visit(tn, w, apex)) return true;
            u = w; w = apex; t = tn;
        }
    }
    return true;
}

// The other subface of facet F holding edge (x,y), given subface (t,f) whose
// third vertex is z; returns t'<<2|f' or -1.
QMD int facet_neighbour(const Mesh& M, int t, int x, int y, int z, int F) {
    int found = -1;
    ring(M, t, x, y, [&](int tt, int u, int w) {
        int4 v = ld4(M.TV, tt);
        int lu = local_of(v, u), lw = local_of(v, w);
        // face opposite u holds (x,y,w); face opposite w holds (x,y,u)
        if (M.TF[4 * (size_t)tt + lu] == F && w != z) { found = (tt << 2) | lu; return true; }
        if (M.TF[4 * (size_t)tt + lw] == F && u != z) { found = (tt << 2) | lw; return true; }
        return false;
    });
    return found;
}

}  // namespace qm
