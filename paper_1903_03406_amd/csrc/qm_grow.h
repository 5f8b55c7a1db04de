// qm_grow.h -- wavefront-cooperative Delaunay-region growth and validation.
//
// One 64-lane wavefront (one workgroup) evaluates one candidate at a time.
// The region is grown breadth-first: each level's (tet, face) pairs are
// spread over the lanes, every lane runs the exact insphere test for its
// neighbour, and new region tets are appended to a work list.  A hash set in
// LDS records every tet tested (inside / outside / claimed), so each tet is
// tested once per candidate.  Work per candidate is proportional to its
// region size, not to one thread per point (the paper's regularised work,
// Section 2).  Regions that outgrow the LDS tiles are re-run from a global
// scratch slab with larger tiles.
#pragma once
#include "qm_kernels.h"

namespace qm {

constexpr unsigned KEYMASK = 0x1FFFFFFFu;
enum { HS_IN = 1u, HS_OUT = 2u, HS_CLAIM = 3u };

struct GrowTiles {
    int* rt; unsigned* H; unsigned* RFH; int* rf; int4* be; unsigned long long* QH; int2* q; int* cx;
    int maxrt, hcap, rfhcap, maxrf, maxbe, qhcap, maxq, maxbf, maxcx;   // cx: 4*maxbf + maxcx ints
};

// boundary-face record written for an accepted candidate (three int4 per face)
//   r0 = (x, y, z, old neighbour)   r1 = (facet id, face flags, ss(x,y), ss(y,z))
//   r2 = (ss(z,x), old tet<<2|face, 0, 0)
struct BfPool { int4* r; int cap; unsigned long long* prof; };   // prof: tested, region, bfaces, claims

struct GrowShared {
    int nrt, nrf, nbf, nbe, nq, ncx, hcount;
    int over, fail, reason;
    int base_reg, base_bf, base_be, base_cl, base_q;
};

QMD unsigned hmix(unsigned k) { return k * 2654435761u; }

// insert key with state; returns 1 inserted, 0 present (old state in *os), -1 full
QMD int hput(unsigned* H, int cap, unsigned key, unsigned state, unsigned* os) {
    unsigned h = hmix(key) & (unsigned)(cap - 1);
    for (int probe = 0; probe < cap; ++probe) {
        unsigned cur = H[h];
        if (cur == 0u) {
            unsigned prev = atomicCAS(&H[h], 0u, key | (state << 29));
            if (prev == 0u) return 1;
            cur = prev;
        }
        if ((cur & KEYMASK) == key) { *os = cur >> 29; return 0; }
        h = (h + 1) & (unsigned)(cap - 1);
    }
    return -1;
}
QMD unsigned hget(const unsigned* H, int cap, unsigned key) {
    unsigned h = hmix(key) & (unsigned)(cap - 1);
    for (int probe = 0; probe < cap; ++probe) {
        unsigned cur = H[h];
        if (cur == 0u) return 0u;
        if ((cur & KEYMASK) == key) return cur >> 29;
        h = (h + 1) & (unsigned)(cap - 1);
    }
    return 0u;
}
// OUT or absent -> CLAIM; returns 1 if this call made the claim
QMD int hclaim(unsigned* H, int cap, unsigned key) {
    unsigned h = hmix(key) & (unsigned)(cap - 1);
    for (int probe = 0; probe < cap; ++probe) {
        unsigned cur = H[h];
        if (cur == 0u) {
            unsigned prev = atomicCAS(&H[h], 0u, key | (HS_CLAIM << 29));
            if (prev == 0u) return 1;
            cur = prev;
        }
        if ((cur & KEYMASK) == key) {
            while ((cur >> 29) == HS_OUT) {
                unsigned prev = atomicCAS(&H[h], cur, key | (HS_CLAIM << 29));
                if (prev == cur) return 1;
                cur = prev;
            }
            return 0;
        }
        h = (h + 1) & (unsigned)(cap - 1);
    }
    return -1;
}
// plain key sets (subfaces of the region)
QMD int sput(unsigned* H, int cap, unsigned key) {
    unsigned h = hmix(key) & (unsigned)(cap - 1);
    for (int probe = 0; probe < cap; ++probe) {
        unsigned cur = H[h];
        if (cur == 0u) {
            unsigned prev = atomicCAS(&H[h], 0u, key);
            if (prev == 0u) return 1;
            cur = prev;
        }
        if (cur == key) return 0;
        h = (h + 1) & (unsigned)(cap - 1);
    }
    return -1;
}
QMD bool shas(const unsigned* H, int cap, unsigned key) {
    unsigned h = hmix(key) & (unsigned)(cap - 1);
    for (int probe = 0; probe < cap; ++probe) {
        unsigned cur = H[h];
        if (cur == 0u) return false;
        if (cur == key) return true;
        h = (h + 1) & (unsigned)(cap - 1);
    }
    return false;
}
QMD int qput(unsigned long long* H, int cap, unsigned long long key) {
    unsigned h = (unsigned)((key * 0x9E3779B97F4A7C15ull) >> 40) & (unsigned)(cap - 1);
    for (int probe = 0; probe < cap; ++probe) {
        unsigned long long cur = H[h];
        if (cur == 0ull) {
            unsigned long long prev = atomicCAS(&H[h], 0ull, key);
            if (prev == 0ull) return 1;
            cur = prev;
        }
        if (cur == key) return 0;
        h = (h + 1) & (unsigned)(cap - 1);
    }
    return -1;
}

QMD double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

// the three vertices of subface (t,f) in ascending order, and edge e of it
// as (x, y, third) in the order (g0,g1), (g0,g2), (g1,g2)
QMD void sub_edge(int4 v, int f, int e, int& x, int& y, int& z) {
    int g0 = at4(v, c_FI[f][0]), g1 = at4(v, c_FI[f][1]), g2 = at4(v, c_FI[f][2]);
    sort3(g0, g1, g2);
    if (e == 0) { x = g0; y = g1; z = g2; }
    else if (e == 1) { x = g0; y = g2; z = g1; }
    else { x = g1; y = g2; z = g0; }
}

// Evaluate candidate `cid` (steps: seeds, grow R_F, grow R_T, validate,
// write results).  All 64 lanes of the workgroup call this together.
__device__ void grow_one(const Mesh& M, int cls, const Cands& C, const Pools& PL, const BfPool& BP,
                         int cid, GrowTiles W, GrowShared& S) {
    const int lane = threadIdx.x;
    const double4 pp = C.p[cid];
    const double P[3] = {pp.x, pp.y, pp.z};
    const int4 tup = C.tup[cid];
    if (lane == 0) {
        S.nrt = S.nrf = S.nbf = S.nbe = S.nq = S.ncx = S.hcount = 0;
        S.over = S.fail = 0; S.reason = EX_NONE;
    }
    for (int i = lane; i < W.hcap; i += 64) W.H[i] = 0u;
    for (int i = lane; i < W.rfhcap; i += 64) W.RFH[i] = 0u;
    for (int i = lane; i < W.qhcap; i += 64) W.QH[i] = 0ull;
    __syncthreads();

    auto add_rt = [&](int t) {
        unsigned os;
        int r = hput(W.H, W.hcap, (unsigned)t + 1u, HS_IN, &os);
        if (r < 0) { S.over = 1; return; }
        if (r == 1) {
            int c = atomicAdd(&S.hcount, 1);
            if (4 * c > 3 * W.hcap) S.over = 1;
            int idx = atomicAdd(&S.nrt, 1);
            if (idx < W.maxrt) W.rt[idx] = t; else S.over = 1;
        }
    };
    auto add_rf = [&](int h) {
        int r = sput(W.RFH, W.rfhcap, (unsigned)face_ckey(M, h >> 2, h & 3) + 1u);
        if (r < 0) { S.over = 1; return; }
        if (r == 1) {
            int idx = atomicAdd(&S.nrf, 1);
            if (idx < W.maxrf && 2 * idx < W.rfhcap) W.rf[idx] = h; else S.over = 1;
        }
    };
    auto in_rf = [&](int t, int f) { return shas(W.RFH, W.rfhcap, (unsigned)face_ckey(M, t, f) + 1u); };

    // ---- seeds
    if (lane == 0) {
        if (cls == CLS_SS) {
            int s = C.elem[cid];
            ring(M, M.STET[s], tup.x, tup.y, [&](int t, int u, int w) {
                add_rt(t);
                int4 v = ld4(M.TV, t);
                int lu = local_of(v, u), lw = local_of(v, w);
                if (M.TF[4 * (size_t)t + lu] >= 0) add_rf((t << 2) | lu);
                if (M.TF[4 * (size_t)t + lw] >= 0) add_rf((t << 2) | lw);
                return false;
            });
        } else if (cls == CLS_SF) {
            add_rf(C.seed[cid]);
        } else {
            add_rt(C.seed[cid]);
        }
    }
    __syncthreads();

    // ---- R_F: subfaces of the seed facets connected across non-subsegment
    // edges whose equatorial ball strictly holds p (seeds always included)
    if (cls != CLS_TET) {
        int head = 0;
        while (true) {
            const int end = S.nrf;
            const bool stop = head >= end || S.over;
            __syncthreads();              // every lane has read the level bounds
            if (stop) break;
            int items = (end - head) * 3;
            for (int k = lane; k < items; k += 64) {
                int h = W.rf[head + k / 3];
                int t = h >> 2, f = h & 3;
                int4 v = ld4(M.TV, t);
                int x, y, z;
                sub_edge(v, f, k % 3, x, y, z);
                if (edge_ss(M, t, v, x, y) >= 0) continue;
                int F = M.TF[4 * (size_t)t + f];
                int nh = facet_neighbour(M, t, x, y, z, F);
                if (nh < 0) continue;
                if (in_rf(nh >> 2, nh & 3)) continue;
                int4 w = ld4(M.TV, nh >> 2);
                int nf = nh & 3;
                double A[3], B[3], Cc[3];
                xyz(M, at4(w, c_FI[nf][0]), A); xyz(M, at4(w, c_FI[nf][1]), B); xyz(M, at4(w, c_FI[nf][2]), Cc);
                if (facedot(A, B, Cc, P) < 0) add_rf(nh);
            }
            __syncthreads();
            head = end;
        }
        // tets on region subfaces are seeds too
        int nrf = S.nrf < W.maxrf ? S.nrf : W.maxrf;
        for (int k = lane; k < nrf; k += 64) {
            int h = W.rf[k];
            add_rt(h >> 2);
            int nb = M.TA[4 * (size_t)(h >> 2) + (h & 3)];
            if (nb >= 0) add_rt(nb >> 2);
        }
        __syncthreads();
    }

    // ---- R_T: tets whose circumsphere strictly holds p, connected to the
    // seeds across faces that are not subfaces (or are region subfaces)
    {
        int head = 0;
        while (true) {
            const int end = S.nrt;
            const bool stop = head >= end || S.over;
            __syncthreads();              // every lane has read the level bounds
            if (stop) break;
            int items = (end - head) * 4;
            for (int k = lane; k < items; k += 64) {
                int t = W.rt[head + (k >> 2)], f = k & 3;
                int nb = M.TA[4 * (size_t)t + f];
                if (nb < 0) continue;
                if (M.TF[4 * (size_t)t + f] >= 0 && !in_rf(t, f)) continue;
                int n = nb >> 2;
                if (n >= M.nt) { atomicOr(&g_geom_error, 64); continue; }
                unsigned key = (unsigned)n + 1u;
                if (hget(W.H, W.hcap, key) != 0u) continue;
                int4 v = ld4(M.TV, n);
                double A[3], B[3], Cc[3], D[3];
                xyz(M, v.x, A); xyz(M, v.y, B); xyz(M, v.z, Cc); xyz(M, v.w, D);
                bool inside = insphere(A, B, Cc, D, P) > 0;
                unsigned os;
                int r = hput(W.H, W.hcap, key, inside ? HS_IN : HS_OUT, &os);
                if (r < 0) { S.over = 1; continue; }
                if (r == 1) {
                    int c = atomicAdd(&S.hcount, 1);
                    if (4 * c > 3 * W.hcap) S.over = 1;
                    if (inside) {
                        int idx = atomicAdd(&S.nrt, 1);
                        if (idx < W.maxrt) W.rt[idx] = n; else S.over = 1;
                    }
                }
            }
            __syncthreads();
            head = end;
        }
    }
    if (S.over) {
        if (lane == 0) C.gst[cid] = ST_OVERFLOW;
        return;
    }
    const int nrt = S.nrt, nrf = S.nrf;
    if (lane == 0 && BP.prof) {
        atomicAdd(&BP.prof[0], (unsigned long long)S.hcount);
        atomicAdd(&BP.prof[1], (unsigned long long)nrt);
    }
    auto in_rt = [&](int t) { return hget(W.H, W.hcap, (unsigned)t + 1u) == HS_IN; };
    auto fail = [&](int reason) { S.fail = 1; S.reason = reason; };   // one reason per phase

    // ---- (a) encroachment: tet points reject on encroached subsegments and
    // subfaces of the region, subface points on subsegments (Shewchuk's rule)
    if (cls != CLS_SS) {
        const int per = cls == CLS_TET ? 10 : 6;
        for (int k = lane; k < nrt * per; k += 64) {
            int t = W.rt[k / per], j = k % per;
            int4 v = ld4(M.TV, t);
            if (j < 6) {
                int s = M.TS[6 * (size_t)t + j];
                if (s < 0) continue;
                double A[3], B[3];
                xyz(M, at4(v, c_EV[j][0]), A); xyz(M, at4(v, c_EV[j][1]), B);
                if (segdot(A, B, P) < 0) {
                    int r = qput(W.QH, W.qhcap, ((unsigned long long)s << 1) + 1ull);
                    if (r == 1) { int idx = atomicAdd(&S.nq, 1); if (idx < W.maxq) W.q[idx] = make_int2(0, s); else S.over = 1; }
                    if (r < 0) S.over = 1;
                }
            } else {
                int f = j - 6;
                if (M.TF[4 * (size_t)t + f] < 0) continue;
                double A[3], B[3], Cc[3];
                xyz(M, at4(v, c_FI[f][0]), A); xyz(M, at4(v, c_FI[f][1]), B); xyz(M, at4(v, c_FI[f][2]), Cc);
                if (facedot(A, B, Cc, P) < 0) {
                    int ck = face_ckey(M, t, f);
                    int r = qput(W.QH, W.qhcap, ((unsigned long long)ck << 1) + 2ull);
                    if (r == 1) { int idx = atomicAdd(&S.nq, 1); if (idx < W.maxq) W.q[idx] = make_int2(1, ck); else S.over = 1; }
                    if (r < 0) S.over = 1;
                }
            }
        }
        __syncthreads();
        if (S.over) {
            if (lane == 0) C.gst[cid] = ST_OVERFLOW;
            return;
        }
        if (S.nq > 0) {
            // rejected: queue the targets, unless all of them are exempt
            __shared__ int any_live;
            if (lane == 0) any_live = 0;
            __syncthreads();
            for (int k = lane; k < S.nq; k += 64) {
                int2 e = W.q[k];
                bool ex = e.x == 0 ? (M.SFL[e.y] & SS_EXEMPT) != 0
                                   : ((M.TI[e.y >> 2] >> (8 + (e.y & 3))) & 1u) != 0;
                if (!ex) any_live = 1;
            }
            __syncthreads();
            if (lane == 0) {
                if (any_live) {
                    int base = atomicAdd(&PL.ctr[4], S.nq);
                    if (base + S.nq > PL.cap_q) { atomicOr(&PL.ctr[5], 1); C.gst[cid] = ST_OVERFLOW; S.base_q = -1; }
                    else { C.gst[cid] = ST_REJECT; C.greason[cid] = EX_NONE; C.q_off[cid] = base; C.q_n[cid] = S.nq; S.base_q = base; }
                } else {
                    C.gst[cid] = ST_EXEMPT; C.greason[cid] = EX_ENC_EXEMPT; S.base_q = -1;
                }
            }
            __syncthreads();
            if (S.base_q >= 0)
                for (int k = lane; k < S.nq; k += 64) PL.q[S.base_q + k] = W.q[k];
            return;
        }
    }

    // ---- (b) insertion radius: nearest region vertex at least h_min away
    {
        double r2 = INFINITY;
        for (int k = lane; k < nrt * 4 + nrf * 3; k += 64) {
            int vid;
            if (k < nrt * 4) vid = M.TV[4 * (size_t)W.rt[k >> 2] + (k & 3)];
            else {
                int j = k - nrt * 4, h = W.rf[j / 3];
                vid = M.TV[4 * (size_t)(h >> 2) + c_FI[h & 3][j % 3]];
            }
            double V[3];
            xyz(M, vid, V);
            double d = d2(V, P);
            if (d < r2) r2 = d;
        }
        r2 = wave_min(r2);
        if (r2 < M.hmin2) {
            if (lane == 0) { C.gst[cid] = ST_EXEMPT; C.greason[cid] = EX_HMIN; }
            return;
        }
    }

    // ---- (c) every tet on a region subface is a region tet
    for (int k = lane; k < nrf; k += 64) {
        int h = W.rf[k];
        int nb = M.TA[4 * (size_t)(h >> 2) + (h & 3)];
        if (!in_rt(h >> 2) || (nb >= 0 && !in_rt(nb >> 2))) fail(EX_RFTET);
    }
    __syncthreads();
    if (S.fail) {
        if (lane == 0) { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; }
        return;
    }

    // ---- (d) boundary faces (not region subfaces; other side hull, outside
    // the region, or a constraint) must see p strictly on their inner side
    for (int k = lane; k < nrt * 4; k += 64) {
        int t = W.rt[k >> 2], f = k & 3;
        int fid = M.TF[4 * (size_t)t + f];
        if (fid >= 0 && in_rf(t, f)) continue;
        int nb = M.TA[4 * (size_t)t + f];
        bool bnd = nb < 0 || !in_rt(nb >> 2) || fid >= 0;
        if (!bnd) continue;
        int4 v = ld4(M.TV, t);
        int x = at4(v, c_FI[f][0]), y = at4(v, c_FI[f][1]), z = at4(v, c_FI[f][2]);
        double A[3], B[3], Cc[3];
        xyz(M, x, A); xyz(M, y, B); xyz(M, z, Cc);
        if (orient3d(A, B, Cc, P) <= 0) { fail(EX_FACE); continue; }
        int idx = atomicAdd(&S.nbf, 1);
        if (idx < W.maxbf) {
            // stage the face record in the claim scratch (x, y, z, neighbour)
            W.cx[4 * idx] = x; W.cx[4 * idx + 1] = y; W.cx[4 * idx + 2] = z; W.cx[4 * idx + 3] = (t << 2) | f;
        } else S.over = 1;
    }
    __syncthreads();
    if (S.over) { if (lane == 0) C.gst[cid] = ST_OVERFLOW; return; }
    if (S.fail) { if (lane == 0) { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; } return; }
    const int nbf = S.nbf;

    // ---- (e) 2D boundary edges of R_F must see p strictly inside, in the
    // facet's projection; the subsegment being split is excluded
    if (cls != CLS_TET) {
        for (int k = lane; k < nrf * 3; k += 64) {
            int h = W.rf[k / 3];
            int t = h >> 2, f = h & 3;
            int4 v = ld4(M.TV, t);
            int x, y, z;
            sub_edge(v, f, k % 3, x, y, z);
            if (cls == CLS_SS && x == tup.x && y == tup.y) continue;
            int F = M.TF[4 * (size_t)t + f];
            bool bnd = edge_ss(M, t, v, x, y) >= 0;
            if (!bnd) {
                int nh = facet_neighbour(M, t, x, y, z, F);
                bnd = nh < 0 || !in_rf(nh >> 2, nh & 3);
            }
            if (!bnd) continue;
            int ax = M.FAX[F];
            double A[3], B[3], Z[3];
            xyz(M, x, A); xyz(M, y, B); xyz(M, z, Z);
            int oz = orient2d(ax, A, B, Z), op = orient2d(ax, A, B, P);
            if (op == 0 || op != oz) { fail(EX_EDGE2D); continue; }
            int one = M.TA[4 * (size_t)t + f] < 0 ? 1 : 0;
            int idx = atomicAdd(&S.nbe, 1);
            if (idx < W.maxbe) W.be[idx] = make_int4(x, y, F, one); else S.over = 1;
        }
        __syncthreads();
        if (S.over) { if (lane == 0) C.gst[cid] = ST_OVERFLOW; return; }
        const int nbe = S.nbe;
        for (int i = lane; i < nbe; i += 64)                  // one new subface per edge
            for (int j = i + 1; j < nbe; ++j)
                if (W.be[i].x == W.be[j].x && W.be[i].y == W.be[j].y) fail(EX_EDGE2D);
        __syncthreads();
        if (S.fail) { if (lane == 0) { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; } return; }
    }
    const int nbe = S.nbe;

    // ---- (f) the boundary closes up around p: each edge of a boundary face
    // lies on two boundary faces (one for a 2D boundary edge of a one-sided
    // region subface); every 2D boundary edge lies on as many
    for (int k = lane; k < nbf * 3 + nbe; k += 64) {
        int x, y;
        if (k < nbf * 3) {
            int i = k / 3, j = k % 3;
            x = W.cx[4 * i + j]; y = W.cx[4 * i + (j + 1) % 3];
        } else {
            int4 e = W.be[k - nbf * 3];
            x = e.x; y = e.y;
        }
        int lo = x < y ? x : y, hi = x < y ? y : x;
        int cnt = 0;
        for (int i = 0; i < nbf; ++i) {
            int a = W.cx[4 * i], b = W.cx[4 * i + 1], c = W.cx[4 * i + 2];
            bool hx = a == x || b == x || c == x, hy = a == y || b == y || c == y;
            cnt += hx && hy;
        }
        int want = 2;
        for (int i = 0; i < nbe; ++i) {
            int4 e = W.be[i];
            if (e.x == lo && e.y == hi && e.w) want = 1;
        }
        if (cnt != want) fail(EX_MANIFOLD);
    }
    __syncthreads();
    if (S.fail) { if (lane == 0) { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; } return; }

    // ---- accepted: claim set = region tets + tets across boundary faces
    int* cext = W.cx + 4 * W.maxbf;              // extra claims after the face records
    for (int i = lane; i < nbf; i += 64) {
        int h = W.cx[4 * i + 3];
        int nb = M.TA[4 * (size_t)(h >> 2) + (h & 3)];
        if (nb < 0) continue;
        int r = hclaim(W.H, W.hcap, (unsigned)(nb >> 2) + 1u);
        if (r == 1) {
            int idx = atomicAdd(&S.ncx, 1);
            if (idx < W.maxcx) cext[idx] = nb >> 2; else S.over = 1;
        } else if (r < 0) S.over = 1;
    }
    __syncthreads();
    if (S.over) { if (lane == 0) C.gst[cid] = ST_OVERFLOW; return; }
    const int ncx = S.ncx;
    if (lane == 0) {
        // region, face and edge pools are only read through this candidate's
        // offsets; the claim pool is scanned whole by the selection, so a
        // claim range is reserved all-or-nothing and only when it will be filled
        int br = atomicAdd(&PL.ctr[0], nrt);
        int bb = atomicAdd(&PL.ctr[1], nbf);
        int be = atomicAdd(&PL.ctr[2], nbe);
        bool full = br + nrt > PL.cap_reg || bb + nbf > PL.cap_bf || bb + nbf > BP.cap ||
                    be + nbe > PL.cap_be;
        int bc = -1;
        if (!full) {
            int cur = atomicAdd(&PL.ctr[3], 0);
            while (true) {
                if (cur + nrt + ncx > PL.cap_cl) { full = true; break; }
                int prev = atomicCAS(&PL.ctr[3], cur, cur + nrt + ncx);
                if (prev == cur) { bc = cur; break; }
                cur = prev;
            }
        }
        if (full) { atomicOr(&PL.ctr[5], 1); C.gst[cid] = ST_OVERFLOW; S.base_reg = -1; }
        else {
            S.base_reg = br; S.base_bf = bb; S.base_be = be; S.base_cl = bc;
            C.reg_off[cid] = br; C.reg_n[cid] = nrt;
            C.bf_off[cid] = bb; C.bf_n[cid] = nbf;
            C.be_off[cid] = be; C.be_n[cid] = nbe;
            C.cl_off[cid] = bc; C.cl_n[cid] = nrt + ncx;
            C.gst[cid] = ST_OK; C.greason[cid] = EX_NONE;
        }
    }
    __syncthreads();
    if (S.base_reg < 0) return;
    if (lane == 0 && BP.prof) {
        atomicAdd(&BP.prof[2], (unsigned long long)nbf);
        atomicAdd(&BP.prof[3], (unsigned long long)(nrt + ncx));
    }
    for (int k = lane; k < nrt; k += 64) {
        PL.reg[S.base_reg + k] = W.rt[k];
        PL.cl[S.base_cl + k] = W.rt[k]; PL.clc[S.base_cl + k] = cid;
    }
    for (int k = lane; k < ncx; k += 64) { PL.cl[S.base_cl + nrt + k] = cext[k]; PL.clc[S.base_cl + nrt + k] = cid; }
    for (int k = lane; k < nbe; k += 64) PL.be[S.base_be + k] = W.be[k];
    for (int i = lane; i < nbf; i += 64) {
        int x = W.cx[4 * i], y = W.cx[4 * i + 1], z = W.cx[4 * i + 2], h = W.cx[4 * i + 3];
        int t = h >> 2, f = h & 3;
        int4 v = ld4(M.TV, t);
        int lx = local_of(v, x), ly = local_of(v, y), lz = local_of(v, z);
        const int* ts = M.TS + 6 * (size_t)t;
        int4 r0 = make_int4(x, y, z, M.TA[4 * (size_t)t + f]);
        int4 r1 = make_int4(M.TF[4 * (size_t)t + f], 0, ts[c_EIDX[lx][ly]], ts[c_EIDX[ly][lz]]);
        int4 r2 = make_int4(ts[c_EIDX[lz][lx]], h, 0, 0);
        BP.r[3 * (size_t)(S.base_bf + i)] = r0;
        BP.r[3 * (size_t)(S.base_bf + i) + 1] = r1;
        BP.r[3 * (size_t)(S.base_bf + i) + 2] = r2;
        PL.bf[S.base_bf + i] = h;
    }
}

template <int MAXRT, int HCAP, int RFHCAP, int MAXRF, int MAXBE, int QHCAP, int MAXQ, int MAXBF>
__global__ __launch_bounds__(64) void k_grow_lds(Mesh M, int cls, Cands C, Pools PL, BfPool BP) {
    __shared__ int rt[MAXRT];
    __shared__ unsigned H[HCAP];
    __shared__ unsigned RFH[RFHCAP];
    __shared__ int rf[MAXRF];
    __shared__ int4 be[MAXBE];
    __shared__ unsigned long long QH[QHCAP];
    __shared__ int2 q[MAXQ];
    __shared__ int cx[4 * MAXBF + MAXBF];
    __shared__ GrowShared S;
    GrowTiles W{rt, H, RFH, rf, be, QH, q, cx, MAXRT, HCAP, RFHCAP, MAXRF, MAXBE, QHCAP, MAXQ, MAXBF, MAXBF};
    for (int cid = blockIdx.x; cid < C.n; cid += gridDim.x) {
        if (C.st[cid] != ST_PENDING) {
            if (threadIdx.x == 0) { C.gst[cid] = C.st[cid]; C.greason[cid] = C.reason[cid]; }
            continue;
        }
        grow_one(M, cls, C, PL, BP, cid, W, S);
        __syncthreads();
    }
}

// re-run of the candidates that overflowed the LDS tiles (or a pool), with
// tiles carved from a global scratch slab; `list` holds their ids
__global__ __launch_bounds__(64) void k_grow_global(Mesh M, int cls, Cands C, Pools PL, BfPool BP,
                                                    const int* list, int nlist, GrowTiles T, char* slab,
                                                    size_t slab_per_block) {
    __shared__ GrowShared S;
    char* base = slab + slab_per_block * blockIdx.x;
    GrowTiles W = T;
    size_t off = 0;
    auto carve = [&](size_t bytes) { char* p = base + off; off += (bytes + 255) & ~(size_t)255; return p; };
    W.rt = (int*)carve(sizeof(int) * T.maxrt);
    W.H = (unsigned*)carve(sizeof(unsigned) * T.hcap);
    W.RFH = (unsigned*)carve(sizeof(unsigned) * T.rfhcap);
    W.rf = (int*)carve(sizeof(int) * T.maxrf);
    W.be = (int4*)carve(sizeof(int4) * T.maxbe);
    W.QH = (unsigned long long*)carve(sizeof(unsigned long long) * T.qhcap);
    W.q = (int2*)carve(sizeof(int2) * T.maxq);
    W.cx = (int*)carve(sizeof(int) * (4 * T.maxbf + T.maxcx));
    for (int i = blockIdx.x; i < nlist; i += gridDim.x) {
        grow_one(M, cls, C, PL, BP, list[i], W, S);
        __syncthreads();
    }
}

inline size_t grow_slab_bytes(const GrowTiles& T) {
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return r(sizeof(int) * T.maxrt) + r(sizeof(unsigned) * T.hcap) + r(sizeof(unsigned) * T.rfhcap) +
           r(sizeof(int) * T.maxrf) + r(sizeof(int4) * T.maxbe) + r(sizeof(unsigned long long) * T.qhcap) +
           r(sizeof(int2) * T.maxq) + r(sizeof(int) * (4 * T.maxbf + T.maxcx));
}

}  // namespace qm
