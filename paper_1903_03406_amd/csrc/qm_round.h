// qm_round.h -- kernels of one round: classify, split, locate, grow and
// validate, flags, selection, insertion.
#pragma once
#include "qm_kernels.h"

namespace qm {

// ------------------------------------------------------------------ classify
// Subsegment ab is encroached when queued, or when a vertex of its link (an
// apex of a tet around ab) lies strictly inside its diametral ball.
// Each classification kernel counts its class in cnt[cls] and writes the
// candidates to cand; a class is skipped when an earlier one has candidates
// (the paper's order), which the kernel reads from cnt itself.
QMD void d_classify_ss(Mesh M, int* cand, int* cnt, const int bid, const int gdim) {
    int s = bid * blockDim.x + threadIdx.x;
    if (s >= M.nss) return;
    int* ncand = cnt + CLS_SS;
    unsigned fl = M.SFL[s];
    if (fl & SS_EXEMPT) return;
    bool enc = (fl & SS_QUEUED) != 0;
    if (!enc && (fl & SS_KNOWN)) enc = (fl & SS_ENC) != 0;   // link unchanged since the last test
    else if (!enc) {
        int2 ab = M.SV[s];
        double A[3], B[3];
        xyz(M, ab.x, A); xyz(M, ab.y, B);
        ring(M, M.STET[s], ab.x, ab.y, [&](int, int u, int w) {
            double V[3];
            xyz(M, u, V);
            if (segdot(A, B, V, M.err) < 0) { enc = true; return true; }
            xyz(M, w, V);
            if (segdot(A, B, V, M.err) < 0) { enc = true; return true; }
            return false;
        });
        M.SFL[s] = fl | SS_KNOWN | (enc ? SS_ENC : 0u);
    }
    if (enc) cand[atomicAdd(ncand, 1)] = s;
}
__global__ void k_classify_ss(Mesh M, int* cand, int* cnt) {
    d_classify_ss(M, cand, cnt, blockIdx.x, gridDim.x);
}

// Subface abc is encroached when queued, or when the apex of one of its
// tets lies strictly inside its equatorial ball.  Each subface is taken from
// the tet whose apex has the smaller id (or its only tet).
QMD void d_classify_sf(Mesh M, int* cand, int* cnt, const int bid, const int gdim) {
    int t = bid * blockDim.x + threadIdx.x;
    if (t >= M.nt || cnt[CLS_SS] > 0) return;
    int* ncand = cnt + CLS_SF;
    unsigned ti = M.TI[t];
    if (!(ti & TI_ALIVE) || !(ti & 0xF0000000u)) return;     // dead, or no subface
    unsigned learnt = 0u;
    for (int f = 0; f < 4; ++f) {
        if (!(ti & ti_fsub(f))) continue;
        bool canon, enc_apex;
        if (ti & ti_fknown(f)) {                               // both apexes unchanged since the test
            canon = (ti & ti_fcanon(f)) != 0;
            enc_apex = (ti & ti_fenc(f)) != 0;
        } else {
            const int4 v = ld4(M.TV, t);
            const int nb = M.TA[4 * (size_t)t + f];
            const int apex2 = nb >= 0 ? M.TV[4 * (size_t)(nb >> 2) + (nb & 3)] : -1;
            canon = !(nb >= 0 && apex2 < at4(v, f));
            enc_apex = false;
            if (canon) {
                double A[3], B[3], C[3], V[3];
                xyz(M, at4(v, c_FI[f][0]), A); xyz(M, at4(v, c_FI[f][1]), B); xyz(M, at4(v, c_FI[f][2]), C);
                xyz(M, at4(v, f), V);
                enc_apex = facedot(A, B, C, V, M.err) < 0;
                if (!enc_apex && apex2 >= 0) { xyz(M, apex2, V); enc_apex = facedot(A, B, C, V, M.err) < 0; }
            }
            learnt |= ti_fknown(f) | (canon ? ti_fcanon(f) : 0u) | (enc_apex ? ti_fenc(f) : 0u);
        }
        if (!canon) continue;                                  // not the canonical copy
        if (ti & (1u << (8 + f))) continue;                    // exempt
        if (enc_apex || (ti & (1u << (4 + f)))) cand[atomicAdd(ncand, 1)] = (t << 2) | f;
    }
    if (learnt) atomicOr(&M.TI[t], learnt);
}
__global__ void k_classify_sf(Mesh M, int* cand, int* cnt) {
    d_classify_sf(M, cand, cnt, blockIdx.x, gridDim.x);
}

// Bad tetrahedron: radius-edge ratio above B (paper, Section 1).
QMD void d_classify_tet(Mesh M, int* cand, int* cnt, const int bid, const int gdim) {
    int t = bid * blockDim.x + threadIdx.x;
    if (t >= M.nt || cnt[CLS_SS] > 0 || cnt[CLS_SF] > 0) return;
    int* ncand = cnt + CLS_TET;
    unsigned ti = M.TI[t];
    if (!(ti & TI_ALIVE) || (ti & TI_EXEMPT)) return;
    if (ti & TI_BADK) {                                        // tested when first classified
        if (ti & TI_BAD) cand[atomicAdd(ncand, 1)] = t;
        return;
    }
    int4 v = ld4(M.TV, t);
    int a = v.x, b = v.y, c = v.z, d = v.w, tmp;
    if (b < a) { tmp = a; a = b; b = tmp; }
    if (d < c) { tmp = c; c = d; d = tmp; }
    if (c < a) { tmp = a; a = c; c = tmp; }
    if (d < b) { tmp = b; b = d; d = tmp; }
    if (c < b) { tmp = b; b = c; c = tmp; }
    double A[3], B[3], C[3], D[3];
    xyz(M, a, A); xyz(M, b, B); xyz(M, c, C); xyz(M, d, D);
    const bool bad = is_bad(A, B, C, D, M.B2);
    atomicOr(&M.TI[t], TI_BADK | (bad ? TI_BAD : 0u));
    if (bad) cand[atomicAdd(ncand, 1)] = t;
}
__global__ void k_classify_tet(Mesh M, int* cand, int* cnt) {
    d_classify_tet(M, cand, cnt, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------ split
// splitting point (paper, Section 2: midpoint / circumcircle centre /
// circumsphere centre) and the predetermined priority of each candidate
// (key_mask: all ones, except in tests that force equal keys)
QMD void d_split(Mesh M, int cls, int n, const int* elem, unsigned long long* key, int4* tup,
                        double4* p, int* st, int* reason, unsigned long long key_mask, const int bid, const int gdim) {
    int i = bid * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int e = elem[i];
    int ids[4] = {-1, -1, -1, -1}, k = 0;
    if (cls == CLS_SS) {
        int2 ab = M.SV[e];
        ids[0] = ab.x; ids[1] = ab.y; k = 2;
    } else if (cls == CLS_SF) {
        int t = e >> 2, f = e & 3;
        int4 v = ld4(M.TV, t);
        ids[0] = at4(v, c_FI[f][0]); ids[1] = at4(v, c_FI[f][1]); ids[2] = at4(v, c_FI[f][2]);
        sort3(ids[0], ids[1], ids[2]);
        k = 3;
    } else {
        int4 v = ld4(M.TV, e);
        ids[0] = v.x; ids[1] = v.y; ids[2] = v.z; ids[3] = v.w;
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b)
                if (ids[b] < ids[a]) { int t = ids[a]; ids[a] = ids[b]; ids[b] = t; }
        k = 4;
    }
    double P[3], V[4][3];
    for (int j = 0; j < k; ++j) xyz(M, ids[j], V[j]);
    if (cls == CLS_SS) midpoint(V[0], V[1], P);
    else if (cls == CLS_SF) tri_cc(V[0], V[1], V[2], P);
    else { double R2; tet_cc(V[0], V[1], V[2], V[3], P, R2); }
    key[i] = prio_key(cls, ids, k) & key_mask;
    tup[i] = make_int4(ids[0], ids[1], ids[2], ids[3]);
    p[i] = make_double4(P[0], P[1], P[2], 0.0);
    bool fin = isfinite(P[0]) && isfinite(P[1]) && isfinite(P[2]);
    st[i] = fin ? ST_PENDING : ST_EXEMPT;
    reason[i] = fin ? EX_NONE : EX_NONFINITE;
}
__global__ void k_split(Mesh M, int cls, int n, const int* elem, unsigned long long* key, int4* tup,
                        double4* p, int* st, int* reason, unsigned long long key_mask) {
    d_split(M, cls, n, elem, key, tup, p, st, reason, key_mask, blockIdx.x, gridDim.x);
}

// order candidates: key descending (radix sort on ~key), equal keys by
// ascending tuple.  Runs of equal keys are rare; one thread fixes each run.
__global__ void k_fix_ties(int n, const unsigned long long* skey, int* order, const int4* tup) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i > 0 && skey[i - 1] == skey[i]) return;           // not the start of a run
    int j = i + 1;
    while (j < n && skey[j] == skey[i]) ++j;
    if (j - i < 2) return;
    for (int a = i + 1; a < j; ++a) {                      // insertion sort of the run
        int x = order[a], b = a - 1;
        int4 tx = tup[x];
        while (b >= i) {
            int4 ty = tup[order[b]];
            bool less = tx.x != ty.x ? tx.x < ty.x : tx.y != ty.y ? tx.y < ty.y
                      : tx.z != ty.z ? tx.z < ty.z : tx.w < ty.w;
            if (!less) break;
            order[b + 1] = order[b]; --b;
        }
        order[b + 1] = x;
    }
}

__global__ void k_permute(int n, const int* order, const int* elem, const unsigned long long* key,
                          const int4* tup, const double4* p, const int* st, const int* reason,
                          Cands C) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int o = order[i];
    C.elem[i] = elem[o]; C.key[i] = key[o]; C.tup[i] = tup[o]; C.p[i] = p[o];
    C.st[i] = st[o]; C.reason[i] = reason[o];
    C.seed[i] = -1; C.qw[i] = make_int2(-1, -1);
}

// ------------------------------------------------------------------ locate
// TET: walk from the bad tet toward p, trying faces by ascending opposite
// vertex id, crossing the first with p strictly outside; crossing a subface
// rejects the point and queues that subface.
// SF: walk on the facet in its 2D projection, edges in ascending order;
// crossing a subsegment rejects the point and queues that subsegment.
QMD void d_locate(Mesh M, int cls, Cands C, const int bid, const int gdim) {
    int i = bid * blockDim.x + threadIdx.x;
    if (i >= C.n || C.st[i] != ST_PENDING) return;
    double4 pp = C.p[i];
    double P[3] = {pp.x, pp.y, pp.z};
    if (cls == CLS_TET) {
        int t = C.elem[i];
        for (int step = 0; step < WALK_CAP; ++step) {
            int4 v = ld4(M.TV, t);
            int ord[4] = {0, 1, 2, 3};
            for (int a = 0; a < 4; ++a)
                for (int b = a + 1; b < 4; ++b)
                    if (at4(v, ord[b]) < at4(v, ord[a])) { int x = ord[a]; ord[a] = ord[b]; ord[b] = x; }
            int next = -1;
            for (int j = 0; j < 4; ++j) {
                int f = ord[j];
                double A[3], B[3], D[3];
                xyz(M, at4(v, c_FI[f][0]), A); xyz(M, at4(v, c_FI[f][1]), B); xyz(M, at4(v, c_FI[f][2]), D);
                if (orient3d_any(A, B, D, P, M.err) >= 0) continue;
                if (M.TF[4 * (size_t)t + f] >= 0) {
                    bool ex = (M.TI[t] >> (8 + f)) & 1u;
                    C.qw[i] = make_int2(1, face_ckey(M, t, f));
                    C.st[i] = ex ? ST_EXEMPT : ST_REJECT;
                    C.reason[i] = ex ? EX_ENC_EXEMPT : EX_NONE;
                    return;
                }
                int nb = M.TA[4 * (size_t)t + f];
                if (nb < 0) { C.st[i] = ST_EXEMPT; C.reason[i] = EX_WALK; return; }
                next = nb >> 2;
                break;
            }
            if (next < 0) { C.seed[i] = t; return; }
            t = next;
        }
        C.st[i] = ST_EXEMPT; C.reason[i] = EX_WALK;
    } else if (cls == CLS_SF) {
        int h = C.elem[i];
        int F = M.TF[4 * (size_t)(h >> 2) + (h & 3)];
        int ax = M.FAX[F];
        for (int step = 0; step < WALK_CAP; ++step) {
            int t = h >> 2, f = h & 3;
            int4 v = ld4(M.TV, t);
            int g0 = at4(v, c_FI[f][0]), g1 = at4(v, c_FI[f][1]), g2 = at4(v, c_FI[f][2]);
            sort3(g0, g1, g2);
            const int E[3][3] = {{g0, g1, g2}, {g0, g2, g1}, {g1, g2, g0}};
            int next = -1;
            for (int j = 0; j < 3; ++j) {
                int x = E[j][0], y = E[j][1], z = E[j][2];
                double Xx[3], Y[3], Z[3];
                xyz(M, x, Xx); xyz(M, y, Y); xyz(M, z, Z);
                int oz = orient2d_any(ax, Xx, Y, Z, M.err);
                int op = orient2d_any(ax, Xx, Y, P, M.err);
                if (op == 0 || op != -oz) continue;
                int s = edge_ss(M, t, v, x, y);
                if (s >= 0) {
                    bool ex = (M.SFL[s] & SS_EXEMPT) != 0;
                    C.qw[i] = make_int2(0, s);
                    C.st[i] = ex ? ST_EXEMPT : ST_REJECT;
                    C.reason[i] = ex ? EX_ENC_EXEMPT : EX_NONE;
                    return;
                }
                next = facet_neighbour(M, t, x, y, z, F);
                if (next < 0) { C.st[i] = ST_EXEMPT; C.reason[i] = EX_WALK; return; }
                break;
            }
            if (next < 0) { C.seed[i] = h; return; }
            h = next;
        }
        C.st[i] = ST_EXEMPT; C.reason[i] = EX_WALK;
    }
}
__global__ void k_locate(Mesh M, int cls, Cands C) {
    d_locate(M, cls, C, blockIdx.x, gridDim.x);
}

}  // namespace qm
