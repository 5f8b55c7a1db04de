// qm_grow.h -- wavefront-cooperative Delaunay-region growth and validation.
//
// One workgroup (one 64-lane wavefront for the common small regions, four
// for the larger tiers) evaluates one candidate at a time.
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
// which tile a region outgrew (GrowShared::over, reported for the largest tiles)
enum { OV_RT = 1, OV_HASH = 2, OV_RF = 4, OV_Q = 8, OV_BF = 16, OV_BE = 32, OV_CX = 64, OV_EDGE = 128 };
enum { HS_IN = 1u, HS_OUT = 2u, HS_CLAIM = 3u };

// Tiles of one candidate's evaluation.  cx (16-byte aligned) holds maxbf
// face records int4 (x, y, z, old tet<<2|face), then 3 ints per face: for the
// edges opposite x, y and z the partner face sharing that edge as m<<2|slot,
// -1 when none; then maxcx extra claims (CXW ints per face in all).  EK/EV: edge table (global-memory tiles only, ehcap
// entries; ehcap 0 selects the pairwise scans bounded by the LDS tiles).
constexpr int CXW = 7;
struct GrowTiles {
    int* rt; unsigned* H; unsigned* RFH; int* rf; int4* be; unsigned long long* QH; int2* q; int* cx;
    int maxrt, hcap, rfhcap, maxrf, maxbe, qhcap, maxq, maxbf, maxcx;
    int tier;             // 0 small LDS tiles, 1 medium LDS tiles, 2 global-memory tiles (the largest)
    unsigned long long* EK; int4* EV; int ehcap;
};

// boundary-face record written for an accepted candidate (BFR int4 per face)
//   r0 = (x, y, z, old neighbour)   r1 = (facet id, face flags, ss(x,y), ss(y,z))
//   r2 = (ss(z,x), old tet<<2|face, 0, 0)
//   r3 = (partner across edge yz, across xz, across xy, 0) as m<<2|slot, m the
//        partner's index among the candidate's faces, -1 on the hull
constexpr int BFR = 4;
// prof: tested, region, bfaces, claims (first small-tile launch); tprof:
// per-tier evaluation counters (every launch), TPROF_W words per tier
struct BfPool { int4* r; int cap; unsigned long long* prof; unsigned long long* tprof; };
constexpr int TPROF_W = 28;   // evals, overflowed, tested, region, bfaces, max region, max tested,
                              // max bfaces, the count of each overflow bit (8), accepted
                              // evaluations and their region tets, boundary faces and claims,
                              // then shader-clock cycles of the 8 phases (lane 0)

// phases timed by ptick: 0 set-up and seeds, 1 R_F, 2 R_T, 3 encroachment,
// 4 insertion radius and R_F tets, 5 boundary faces, 6 2D edges and closure,
// 7 claims and results
constexpr int GROW_PHASES = 8;
struct GrowShared {
    int nrt, nrf, nbf, nbe, nq, ncx, hcount;
    int over, fail, reason, accepted, lost;
    int base_reg, base_bf, base_be, base_cl, base_q;
    int take;                                   // next candidate of a shared-counter loop
    unsigned long long prof[4 + GROW_PHASES];   // region counters and phase clocks of this workgroup
    unsigned long long tlast;                   // (flushed at exit)
};

QMD void prof_begin(GrowShared& S) {
    if (threadIdx.x == 0)
        for (int i = 0; i < 4 + GROW_PHASES; ++i) S.prof[i] = 0ull;
}
// profiling: one finished evaluation of tier `tier` (lane 0, after grow_one)
QMD void tier_count(const GrowShared& S, const BfPool& BP, int tier) {
    if (threadIdx.x != 0 || !BP.tprof) return;
    unsigned long long* c = BP.tprof + TPROF_W * tier;
    atomicAdd(&c[0], 1ull);
    if (S.over) {
        atomicAdd(&c[1], 1ull);
        for (int b = 0; b < 8; ++b)
            if (S.over & (1 << b)) atomicAdd(&c[8 + b], 1ull);
        return;
    }
    atomicAdd(&c[2], (unsigned long long)S.hcount);
    atomicAdd(&c[3], (unsigned long long)S.nrt);
    atomicAdd(&c[4], (unsigned long long)S.nbf);
    atomicMax(&c[5], (unsigned long long)S.nrt);
    atomicMax(&c[6], (unsigned long long)S.hcount);
    atomicMax(&c[7], (unsigned long long)S.nbf);
    if (S.accepted) {
        atomicAdd(&c[16], 1ull);
        atomicAdd(&c[17], (unsigned long long)S.nrt);
        atomicAdd(&c[18], (unsigned long long)S.nbf);
        atomicAdd(&c[19], (unsigned long long)(S.nrt + S.ncx));
    }
}
QMD void prof_flush(const GrowShared& S, const BfPool& BP, int tier) {
    if (threadIdx.x == 0 && BP.prof)
        for (int i = 0; i < 4 + GROW_PHASES; ++i)
            if (S.prof[i]) atomicAdd(&BP.prof[i], S.prof[i]);
    if (threadIdx.x == 0 && BP.tprof)
        for (int i = 0; i < GROW_PHASES; ++i)
            if (S.prof[4 + i]) atomicAdd(&BP.tprof[TPROF_W * tier + 20 + i], S.prof[4 + i]);
}
// shader clock at a phase boundary (profiling only): the cycles since the
// last boundary go to phase `ph`
QMD void ptick(GrowShared& S, const BfPool& BP, int ph) {
    if ((BP.prof || BP.tprof) && threadIdx.x == 0) {
        unsigned long long t = clock64();
        if (ph >= 0) S.prof[4 + ph] += t - S.tlast;
        S.tlast = t;
    }
}

// End of a validation phase: wait for every lane's writes, take the verdict
// flags, and wait again so that no lane starts the next phase (which may
// set the flags) before all have read them.  True: stop (over or failed).
QMD bool phase_end(const GrowShared& S) {
    __syncthreads();
    const bool stop = S.over != 0 || S.fail != 0 || S.lost != 0;
    __syncthreads();
    return stop;
}

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

// edge table of the global-memory tiles: key (lo<<32 | hi) with bit 63 set,
// value (faces holding the edge, first and second face-edge code, 2D
// boundary edges with this key + 0x10000 if one of them is one-sided)
QMD unsigned long long ekey(int x, int y) {
    unsigned lo = (unsigned)(x < y ? x : y), hi = (unsigned)(x < y ? y : x);
    return ((unsigned long long)lo << 32) | hi | (1ull << 63);
}
QMD unsigned ehash(unsigned long long k, int cap) {
    return (unsigned)((k * 0x9E3779B97F4A7C15ull) >> 40) & (unsigned)(cap - 1);
}
QMD int eput(unsigned long long* EK, int cap, unsigned long long key) {   // slot of key (inserted)
    unsigned h = ehash(key, cap);
    for (int probe = 0; probe < cap; ++probe) {
        unsigned long long cur = EK[h];
        if (cur == 0ull) {
            unsigned long long prev = atomicCAS(&EK[h], 0ull, key);
            if (prev == 0ull) return (int)h;
            cur = prev;
        }
        if (cur == key) return (int)h;
        h = (h + 1) & (unsigned)(cap - 1);
    }
    return -1;
}
QMD int eget(const unsigned long long* EK, int cap, unsigned long long key) {   // slot or -1
    unsigned h = ehash(key, cap);
    for (int probe = 0; probe < cap; ++probe) {
        unsigned long long cur = EK[h];
        if (cur == 0ull) return -1;
        if (cur == key) return (int)h;
        h = (h + 1) & (unsigned)(cap - 1);
    }
    return -1;
}
// table size for n keys (power of two, at least 2n), cleared by all NT lanes
template <int NT> QMD int eclear(const GrowTiles& W, int n) {
    int cap = 64;
    while (cap < 2 * n) cap <<= 1;
    if (cap > W.ehcap) cap = W.ehcap;
    for (int i = threadIdx.x; i < cap; i += NT) { W.EK[i] = 0ull; W.EV[i] = make_int4(0, -1, -1, 0); }
    return cap;
}

QMD double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
// minimum over the NT lanes of the workgroup (every lane gets it)
template <int NT> QMD double block_min(double v) {
    v = wave_min(v);
    if (NT == 64) return v;
    __shared__ double part[NT / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = part[0];
    for (int i = 1; i < NT / 64; ++i) r = fmin(r, part[i]);
    __syncthreads();
    return r;
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

// a region over the tiles: evaluate again with the next tier's tiles, or
// (largest tiles) report which tile was too small in the counter word
// PL.ctr[35].  A bad tet remembers the tier its region needed (bits 12-13 of
// its info word: 1 medium, 3 global) so that its evaluations in later
// rounds start there; the word is rewritten when the slot gets a new tet.
QMD void over_status(const Mesh& M, int cls, const Cands& C, const Pools& PL, const GrowTiles& W, int cid,
                     int over, const GrowShared& S) {
    if (cls == CLS_TET && W.tier < 2) atomicOr(&M.TI[C.elem[cid]], (W.tier == 0 ? 1u : 3u) << TI_HINT_SHIFT);
    if (W.tier == 2) {
        C.gst[cid] = ST_TOOBIG;
        atomicOr(&PL.ctr[35], over);
        atomicMax(&PL.ctr[44], S.nrt);       // largest region and tested count reached
        atomicMax(&PL.ctr[45], S.hcount);
    } else C.gst[cid] = W.tier == 0 ? ST_OVERFLOW : ST_OVERFLOW2;
}

// results that did not fit a pool: the whole pass is evaluated again with
// larger pools
QMD int poolfull_status(const GrowTiles&) { return ST_POOLFULL; }

// Evaluate candidate `cid` (steps: seeds, grow R_F, grow R_T, validate,
// write results).  All NT lanes of the workgroup call this together.
template <int NT>
__device__ void grow_one(const Mesh& M, int cls, const Cands& C, const Pools& PL, const BfPool& BP,
                         int cid, GrowTiles W, GrowShared& S) {
    const int lane = threadIdx.x;
    const double4 pp = C.p[cid];
    const double P[3] = {pp.x, pp.y, pp.z};
    const int4 tup = C.tup[cid];
    int4* const CF = reinterpret_cast<int4*>(W.cx);       // boundary-face records
    int* const CP = W.cx + 4 * W.maxbf;                     // their edge partners
    ptick(S, BP, -1);
    if (lane == 0) {
        S.nrt = S.nrf = S.nbf = S.nbe = S.nq = S.ncx = S.hcount = 0;
        S.over = S.fail = 0; S.reason = EX_NONE; S.accepted = 0; S.lost = 0;
    }
    for (int i = lane; i < W.hcap; i += NT) W.H[i] = 0u;
    for (int i = lane; i < W.rfhcap; i += NT) W.RFH[i] = 0u;
    for (int i = lane; i < W.qhcap; i += NT) W.QH[i] = 0ull;
    __syncthreads();

    // Early-stop blasting (non-parity mode, Section 2's blasting as the paper
    // runs it): every tet the candidate takes is marked with its priority in
    // this pass; meeting a mark of higher priority stops the candidate, which
    // waits for a later round.
    const unsigned long long es_v =
        ((unsigned long long)PL.es_pass << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)cid);
    auto es_take = [&](int t) {
        if (PL.es_mark && atomicMax(&PL.es_mark[t], es_v) > es_v) S.lost = 1;
    };
    auto add_rt = [&](int t) {
        unsigned os;
        int r = hput(W.H, W.hcap, (unsigned)t + 1u, HS_IN, &os);
        if (r < 0) { S.over |= OV_HASH; return; }
        if (r == 1) {
            es_take(t);
            int c = atomicAdd(&S.hcount, 1);
            if (4 * c > 3 * W.hcap) S.over |= OV_HASH;
            int idx = atomicAdd(&S.nrt, 1);
            if (idx < W.maxrt) W.rt[idx] = t; else S.over |= OV_RT;
        }
    };
    auto add_rf = [&](int h) {
        int r = sput(W.RFH, W.rfhcap, (unsigned)face_ckey(M, h >> 2, h & 3) + 1u);
        if (r < 0) { S.over |= OV_RF; return; }
        if (r == 1) {
            int idx = atomicAdd(&S.nrf, 1);
            if (idx < W.maxrf && 2 * idx < W.rfhcap) W.rf[idx] = h; else S.over |= OV_RF;
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
    ptick(S, BP, 0);

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
            for (int k = lane; k < items; k += NT) {
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
                if (facedot(A, B, Cc, P, M.err) < 0) add_rf(nh);
            }
            __syncthreads();
            head = end;
        }
        // tets on region subfaces are seeds too
        int nrf = S.nrf < W.maxrf ? S.nrf : W.maxrf;
        for (int k = lane; k < nrf; k += NT) {
            int h = W.rf[k];
            add_rt(h >> 2);
            int nb = M.TA[4 * (size_t)(h >> 2) + (h & 3)];
            if (nb >= 0) add_rt(nb >> 2);
        }
        __syncthreads();
    }

    ptick(S, BP, 1);
    // ---- R_T: tets whose circumsphere strictly holds p, connected to the
    // seeds across faces that are not subfaces (or are region subfaces)
    bool over_rt = false;
    {
        int head = 0;
        while (true) {
            const int end = S.nrt;
            over_rt = S.over != 0 || S.lost != 0;
            const bool stop = head >= end || over_rt;
            __syncthreads();              // every lane has read the level bounds
            if (stop) break;
            int items = (end - head) * 4;
            for (int k = lane; k < items; k += NT) {
                int t = W.rt[head + (k >> 2)], f = k & 3;
                int nb = M.TA[4 * (size_t)t + f];
                if (nb < 0) continue;
                if (M.TF[4 * (size_t)t + f] >= 0 && !in_rf(t, f)) continue;
                int n = nb >> 2;
                if (n >= M.nt) { atomicOr(M.err, 64); continue; }
                unsigned key = (unsigned)n + 1u;
                if (hget(W.H, W.hcap, key) != 0u) continue;
                int4 v = ld4(M.TV, n);
                double A[3], B[3], Cc[3], D[3];
                xyz(M, v.x, A); xyz(M, v.y, B); xyz(M, v.z, Cc); xyz(M, v.w, D);
                bool inside = insphere(A, B, Cc, D, P, M.err) > 0;
                unsigned os;
                int r = hput(W.H, W.hcap, key, inside ? HS_IN : HS_OUT, &os);
                if (r < 0) { S.over |= OV_HASH; continue; }
                if (r == 1) {
                    int c = atomicAdd(&S.hcount, 1);
                    if (4 * c > 3 * W.hcap) S.over |= OV_HASH;
                    if (inside) {
                        es_take(n);
                        int idx = atomicAdd(&S.nrt, 1);
                        if (idx < W.maxrt) W.rt[idx] = n; else S.over |= OV_RT;
                    }
                }
            }
            __syncthreads();
            head = end;
        }
    }
    if (over_rt) {                        // read before the last level barrier
        if (lane == 0) {
            if (S.lost) C.gst[cid] = ST_LOST;
            else over_status(M, cls, C, PL, W, cid, S.over, S);
        }
        return;
    }
    const int nrt = S.nrt, nrf = S.nrf;
    if (lane == 0) { S.prof[0] += S.hcount; S.prof[1] += nrt; }
    ptick(S, BP, 2);
    auto in_rt = [&](int t) { return hget(W.H, W.hcap, (unsigned)t + 1u) == HS_IN; };
    auto fail = [&](int reason) { S.fail = 1; S.reason = reason; };   // one reason per phase

    // ---- (a) encroachment: tet points reject on encroached subsegments and
    // subfaces of the region, subface points on subsegments (Shewchuk's rule)
    if (cls != CLS_SS) {
        // one region tet per lane: its six edge words and (tet points) four
        // face words are loaded together; most are not constraints
        for (int k = lane; k < nrt; k += NT) {
            const int t = W.rt[k];
            const int* ts = M.TS + 6 * (size_t)t;
            const int s6[6] = {ts[0], ts[1], ts[2], ts[3], ts[4], ts[5]};
            const int4 tf = cls == CLS_TET ? ld4(M.TF, t) : make_int4(-1, -1, -1, -1);
            // the AND of the words has its sign bit clear iff some word is >= 0
            if ((s6[0] & s6[1] & s6[2] & s6[3] & s6[4] & s6[5] & tf.x & tf.y & tf.z & tf.w) < 0) continue;
            const int4 v = ld4(M.TV, t);
            for (int j = 0; j < 6; ++j) {
                const int s = s6[j];
                if (s < 0) continue;
                double A[3], B[3];
                xyz(M, at4(v, c_EV[j][0]), A); xyz(M, at4(v, c_EV[j][1]), B);
                if (segdot(A, B, P, M.err) < 0) {
                    int r = qput(W.QH, W.qhcap, ((unsigned long long)s << 1) + 1ull);
                    if (r == 1) { int idx = atomicAdd(&S.nq, 1); if (idx < W.maxq) W.q[idx] = make_int2(0, s); else S.over |= OV_Q; }
                    if (r < 0) S.over |= OV_Q;
                }
            }
            for (int f = 0; f < 4; ++f) {
                if (at4(tf, f) < 0) continue;
                double A[3], B[3], Cc[3];
                xyz(M, at4(v, c_FI[f][0]), A); xyz(M, at4(v, c_FI[f][1]), B); xyz(M, at4(v, c_FI[f][2]), Cc);
                if (facedot(A, B, Cc, P, M.err) < 0) {
                    int ck = face_ckey(M, t, f);
                    int r = qput(W.QH, W.qhcap, ((unsigned long long)ck << 1) + 2ull);
                    if (r == 1) { int idx = atomicAdd(&S.nq, 1); if (idx < W.maxq) W.q[idx] = make_int2(1, ck); else S.over |= OV_Q; }
                    if (r < 0) S.over |= OV_Q;
                }
            }
        }
        __syncthreads();
        const bool over_q = S.over != 0;
        const int nq = S.nq;
        __syncthreads();                  // flags read before any lane goes on
        if (over_q) {
            if (lane == 0) over_status(M, cls, C, PL, W, cid, S.over, S);
            return;
        }
        if (nq > 0) {
            // rejected: queue the targets, unless all of them are exempt
            __shared__ int any_live;
            if (lane == 0) any_live = 0;
            __syncthreads();
            for (int k = lane; k < S.nq; k += NT) {
                int2 e = W.q[k];
                bool ex = e.x == 0 ? (M.SFL[e.y] & SS_EXEMPT) != 0
                                   : ((M.TI[e.y >> 2] >> (8 + (e.y & 3))) & 1u) != 0;
                if (!ex) any_live = 1;
            }
            __syncthreads();
            if (lane == 0) {
                if (any_live) {
                    int base = atomicAdd(&PL.ctr[4], S.nq);
                    if (base + S.nq > PL.cap_q) { atomicOr(&PL.ctr[5], 1); C.gst[cid] = poolfull_status(W); S.base_q = -1; }
                    else { C.gst[cid] = ST_REJECT; C.greason[cid] = EX_NONE; C.q_off[cid] = base; C.q_n[cid] = S.nq; S.base_q = base; }
                } else {
                    C.gst[cid] = ST_EXEMPT; C.greason[cid] = EX_ENC_EXEMPT; S.base_q = -1;
                }
            }
            __syncthreads();
            if (S.base_q >= 0)
                for (int k = lane; k < S.nq; k += NT) PL.q[S.base_q + k] = W.q[k];
            return;
        }
    }

    ptick(S, BP, 3);
    // ---- (b) insertion radius: nearest region vertex at least h_min away
    {
        double r2 = INFINITY;
        for (int k = lane; k < nrt + nrf * 3; k += NT) {
            if (k < nrt) {                       // the four vertices of a region tet
                const int4 v = ld4(M.TV, W.rt[k]);
                double V0[3], V1[3], V2[3], V3[3];
                xyz(M, v.x, V0); xyz(M, v.y, V1); xyz(M, v.z, V2); xyz(M, v.w, V3);
                r2 = fmin(r2, fmin(fmin(d2(V0, P), d2(V1, P)), fmin(d2(V2, P), d2(V3, P))));
            } else {                             // a vertex of a region subface
                int j = k - nrt, h = W.rf[j / 3];
                double V[3];
                xyz(M, M.TV[4 * (size_t)(h >> 2) + c_FI[h & 3][j % 3]], V);
                r2 = fmin(r2, d2(V, P));
            }
        }
        r2 = block_min<NT>(r2);
        if (r2 < M.hmin2) {
            if (lane == 0) { C.gst[cid] = ST_EXEMPT; C.greason[cid] = EX_HMIN; }
            return;
        }
    }

    // ---- (c) every tet on a region subface is a region tet
    for (int k = lane; k < nrf; k += NT) {
        int h = W.rf[k];
        int nb = M.TA[4 * (size_t)(h >> 2) + (h & 3)];
        if (!in_rt(h >> 2) || (nb >= 0 && !in_rt(nb >> 2))) fail(EX_RFTET);
    }
    if (phase_end(S)) {
        if (lane == 0) { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; }
        return;
    }

    ptick(S, BP, 4);
    // ---- (d) boundary faces (not region subfaces; other side hull, outside
    // the region, or a constraint) must see p strictly on their inner side
    for (int k = lane; k < nrt; k += NT) {      // one region tet per lane, its four faces
        const int t = W.rt[k];
        const int4 tf = ld4(M.TF, t), ta = ld4(M.TA, t), v = ld4(M.TV, t);
        for (int f = 0; f < 4; ++f) {
            const int fid = at4(tf, f);
            if (fid >= 0 && in_rf(t, f)) continue;
            const int nb = at4(ta, f);
            const bool bnd = nb < 0 || fid >= 0 || !in_rt(nb >> 2);
            if (!bnd) continue;
            const int x = at4(v, c_FI[f][0]), y = at4(v, c_FI[f][1]), z = at4(v, c_FI[f][2]);
            double A[3], B[3], Cc[3];
            xyz(M, x, A); xyz(M, y, B); xyz(M, z, Cc);
            if (orient3d(A, B, Cc, P, M.err) <= 0) { fail(EX_FACE); continue; }
            int idx = atomicAdd(&S.nbf, 1);
            if (idx < W.maxbf) {
                // stage the face record in the claim scratch (x, y, z, old tet<<2|face)
                reinterpret_cast<int4*>(W.cx)[idx] = make_int4(x, y, z, (t << 2) | f);
            } else S.over |= OV_BF;
        }
    }
    if (phase_end(S)) {
        if (lane == 0) {
            if (S.over) over_status(M, cls, C, PL, W, cid, S.over, S);
            else { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; }
        }
        return;
    }
    const int nbf = S.nbf;

    ptick(S, BP, 5);
    // ---- (e) 2D boundary edges of R_F must see p strictly inside, in the
    // facet's projection; the subsegment being split is excluded
    if (cls != CLS_TET) {
        for (int k = lane; k < nrf * 3; k += NT) {
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
            int oz = orient2d(ax, A, B, Z, M.err), op = orient2d(ax, A, B, P, M.err);
            if (op == 0 || op != oz) { fail(EX_EDGE2D); continue; }
            int one = M.TA[4 * (size_t)t + f] < 0 ? 1 : 0;
            int idx = atomicAdd(&S.nbe, 1);
            if (idx < W.maxbe) W.be[idx] = make_int4(x, y, F, one); else S.over |= OV_BE;
        }
        if (phase_end(S)) {
            if (lane == 0) {
                if (S.over) over_status(M, cls, C, PL, W, cid, S.over, S);
                else { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; }
            }
            return;
        }
        const int nbe = S.nbe;
        // one new subface per edge: no two 2D boundary edges alike
        if (W.ehcap) {
            const int ecap = eclear<NT>(W, 3 * nbf + nbe);
            __syncthreads();
            for (int i = lane; i < nbe; i += NT) {
                int4 e = W.be[i];
                int sl = eput(W.EK, ecap, ekey(e.x, e.y));
                if (sl < 0) { S.over |= OV_EDGE; continue; }
                atomicAdd(&W.EV[sl].w, 1 + (e.w ? 0x10000 : 0));
            }
            __syncthreads();
            for (int i = lane; i < nbe; i += NT) {
                int4 e = W.be[i];
                int sl = eget(W.EK, ecap, ekey(e.x, e.y));
                if (sl >= 0 && (W.EV[sl].w & 0xFFFF) > 1) fail(EX_EDGE2D);
            }
        } else {
            for (int i = lane; i < nbe; i += NT)
                for (int j = i + 1; j < nbe; ++j)
                    if (W.be[i].x == W.be[j].x && W.be[i].y == W.be[j].y) fail(EX_EDGE2D);
        }
        if (phase_end(S)) {
            if (lane == 0) {
                if (S.over) over_status(M, cls, C, PL, W, cid, S.over, S);
                else { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; }
            }
            return;
        }
    } else if (W.ehcap) {
        eclear<NT>(W, 3 * nbf);
    }
    const int nbe = S.nbe;

    // ---- (f) the boundary closes up around p: each edge of a boundary face
    // lies on two boundary faces (one for a 2D boundary edge of a one-sided
    // region subface); every 2D boundary edge lies on as many.  The face
    // sharing each edge is recorded: it is the neighbour of the new tet.
    // Edge of face i opposite its slot l: l = 0 (y,z), 1 (x,z), 2 (x,y).
    if (W.ehcap) {
        int ecap = 64;
        while (ecap < 2 * (3 * nbf + nbe)) ecap <<= 1;
        if (ecap > W.ehcap) ecap = W.ehcap;
        __syncthreads();                  // table cleared (and 2D boundary edges in)
        for (int k = lane; k < 3 * nbf; k += NT) {
            const int i = k / 3, l = k % 3;
            const int4 r = CF[i];
            int sl = eput(W.EK, ecap, ekey(l == 0 ? r.y : r.x, l == 2 ? r.y : r.z));
            if (sl < 0) { S.over |= OV_EDGE; continue; }
            atomicAdd(&W.EV[sl].x, 1);
            const int fe = (i << 2) | l;
            if (atomicCAS(&W.EV[sl].y, -1, fe) != -1) atomicCAS(&W.EV[sl].z, -1, fe);
        }
        __syncthreads();
        for (int k = lane; k < 3 * nbf + nbe; k += NT) {
            unsigned long long key;
            if (k < 3 * nbf) {
                const int4 r = CF[k / 3];
                const int l = k % 3;
                key = ekey(l == 0 ? r.y : r.x, l == 2 ? r.y : r.z);
            } else {
                int4 e = W.be[k - 3 * nbf];
                key = ekey(e.x, e.y);
            }
            int sl = eget(W.EK, ecap, key);
            int4 ev = sl >= 0 ? W.EV[sl] : make_int4(0, -1, -1, 0);
            int want = (ev.w & 0x10000) ? 1 : 2;
            if (ev.x != want) { fail(EX_MANIFOLD); continue; }
            if (k < 3 * nbf) {
                const int fe = ((k / 3) << 2) | (k % 3);
                CP[3 * (k / 3) + k % 3] = want == 1 ? -1 : (ev.y == fe ? ev.z : ev.y);
            }
        }
    } else {
        for (int k = lane; k < 3 * nbf + nbe; k += NT) {
            int u, w, i = -1, l = 0;
            if (k < 3 * nbf) {
                i = k / 3; l = k % 3;
                const int4 r = CF[i];
                u = l == 0 ? r.y : r.x;
                w = l == 2 ? r.y : r.z;
            } else {
                int4 e = W.be[k - 3 * nbf];
                u = e.x; w = e.y;
            }
            int cnt = 0, partner = -1;
            for (int m = 0; m < nbf; ++m) {
                const int4 q = CF[m];
                bool hu = q.x == u || q.y == u || q.z == u, hw = q.x == w || q.y == w || q.z == w;
                if (hu && hw) {
                    ++cnt;
                    if (m != i) partner = (m << 2) | ((q.x != u && q.x != w) ? 0 : ((q.y != u && q.y != w) ? 1 : 2));
                }
            }
            const int lo = u < w ? u : w, hi = u < w ? w : u;
            int want = 2;
            for (int j = 0; j < nbe; ++j) {
                int4 e = W.be[j];
                if (e.x == lo && e.y == hi && e.w) want = 1;
            }
            if (cnt != want) { fail(EX_MANIFOLD); continue; }
            if (i >= 0) CP[3 * i + l] = want == 1 ? -1 : partner;
        }
    }
    if (phase_end(S)) {
        if (lane == 0) {
            if (S.over) over_status(M, cls, C, PL, W, cid, S.over, S);
            else { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; }
        }
        return;
    }

    // ---- (g) the mesh stays a CDT (every round ends with one, Section 2):
    // each new interior face (u, w, p) that is not a new subface lies between
    // the new tets on the two boundary faces holding edge uw; it must be
    // locally Delaunay, i.e. the partner face's third vertex is not strictly
    // inside the circumsphere of (x, y, z, p), positively oriented by (d).
    // The two new tets give the same sign, so each pair is tested once.
    {
        int ecap = 64;
        while (ecap < 2 * (3 * nbf + nbe)) ecap <<= 1;
        if (ecap > W.ehcap) ecap = W.ehcap;
        for (int k = lane; k < 3 * nbf; k += NT) {
            const int pr = CP[k];
            const int i = k / 3, l = k % 3;
            if (pr < 0 || (pr >> 2) < i) continue;
            const int4 r = CF[i];
            const int u = l == 0 ? r.y : r.x, w = l == 2 ? r.y : r.z;
            bool sub = false;                    // uw is a 2D boundary edge: (u, w, p) is a subface
            if (nbe > 0) {
                if (W.ehcap) {
                    const int sl = eget(W.EK, ecap, ekey(u, w));
                    sub = sl >= 0 && (W.EV[sl].w & 0xFFFF) > 0;
                } else {
                    const int lo = u < w ? u : w, hi = u < w ? w : u;
                    for (int j = 0; j < nbe && !sub; ++j) sub = W.be[j].x == lo && W.be[j].y == hi;
                }
            }
            if (sub) continue;
            const int apex = at4(CF[pr >> 2], pr & 3);
            double A[3], B[3], Cc[3], Q[3];
            xyz(M, r.x, A); xyz(M, r.y, B); xyz(M, r.z, Cc); xyz(M, apex, Q);
            if (insphere(A, B, Cc, P, Q, M.err) > 0) fail(EX_DELAUNAY);
        }
        if (phase_end(S)) {
            if (lane == 0) { C.gst[cid] = ST_EXEMPT; C.greason[cid] = S.reason; }
            return;
        }
    }

    ptick(S, BP, 6);
    // ---- accepted: claim set = region tets + tets across boundary faces
    int* cext = W.cx + CXW * W.maxbf;            // extra claims after the face records
    for (int i = lane; i < nbf; i += NT) {
        int h = CF[i].w;
        int nb = M.TA[4 * (size_t)(h >> 2) + (h & 3)];
        if (nb < 0) continue;
        int r = hclaim(W.H, W.hcap, (unsigned)(nb >> 2) + 1u);
        if (r == 1) {
            es_take(nb >> 2);
            int idx = atomicAdd(&S.ncx, 1);
            if (idx < W.maxcx) cext[idx] = nb >> 2; else S.over |= OV_CX;
        } else if (r < 0) S.over |= OV_HASH;
    }
    if (phase_end(S)) {
        if (lane == 0) {
            if (S.lost) C.gst[cid] = ST_LOST;
            else over_status(M, cls, C, PL, W, cid, S.over, S);
        }
        return;
    }
    const int ncx = S.ncx;
    if (lane == 0) {
        // face and edge pools are only read through this candidate's offsets;
        // the claim pool is scanned whole by the selection, so a reserved
        // claim range that will not be filled is marked void (-1).  The claim
        // range starts with the region tets, which is also the region list.
        int bb = atomicAdd(&PL.ctr[1], nbf);
        int be = nbe > 0 ? atomicAdd(&PL.ctr[2], nbe) : 0;
        int bc = atomicAdd(&PL.ctr[3], nrt + ncx);
        bool full = bb + nbf > BP.cap || be + nbe > PL.cap_be || bc + nrt + ncx > PL.cap_cl;
        if (full) {
            atomicOr(&PL.ctr[5], 1); C.gst[cid] = poolfull_status(W); S.base_reg = -1;
            S.base_cl = bc;
        } else {
            S.base_reg = bc; S.base_bf = bb; S.base_be = be; S.base_cl = bc;
            C.reg_off[cid] = bc; C.reg_n[cid] = nrt;
            C.bf_off[cid] = bb; C.bf_n[cid] = nbf;
            C.be_off[cid] = be; C.be_n[cid] = nbe;
            C.cl_off[cid] = bc; C.cl_n[cid] = nrt + ncx;
            C.gst[cid] = ST_OK; C.greason[cid] = EX_NONE;
            S.accepted = 1;
        }
    }
    __syncthreads();
    if (S.base_reg < 0) {
        const int end = S.base_cl + nrt + ncx < PL.cap_cl ? S.base_cl + nrt + ncx : PL.cap_cl;
        for (int k = S.base_cl + lane; k < end; k += NT) PL.clc[k] = -1;
        return;
    }
    if (lane == 0) { S.prof[2] += nbf; S.prof[3] += nrt + ncx; }
    for (int k = lane; k < nrt; k += NT) { PL.cl[S.base_cl + k] = W.rt[k]; PL.clc[S.base_cl + k] = cid; }
    for (int k = lane; k < ncx; k += NT) { PL.cl[S.base_cl + nrt + k] = cext[k]; PL.clc[S.base_cl + nrt + k] = cid; }
    for (int k = lane; k < nbe; k += NT) PL.be[S.base_be + k] = W.be[k];
    for (int i = lane; i < nbf; i += NT) {
        const int4 rc = CF[i];
        const int* pc = CP + 3 * i;
        int x = rc.x, y = rc.y, z = rc.z, h = rc.w;
        int t = h >> 2, f = h & 3;
        int4 v = ld4(M.TV, t);
        int lx = local_of(v, x), ly = local_of(v, y), lz = local_of(v, z);
        const int* ts = M.TS + 6 * (size_t)t;
        int4 r0 = make_int4(x, y, z, M.TA[4 * (size_t)t + f]);
        int4 r1 = make_int4(M.TF[4 * (size_t)t + f], 0, ts[c_EIDX[lx][ly]], ts[c_EIDX[ly][lz]]);
        int4 r2 = make_int4(ts[c_EIDX[lz][lx]], h, 0, 0);
        int4* out = BP.r + BFR * (size_t)(S.base_bf + i);
        out[0] = r0; out[1] = r1; out[2] = r2; out[3] = make_int4(pc[0], pc[1], pc[2], 0);
    }
    ptick(S, BP, 7);
}

// LDS tiles; TIER 1 (medium) also takes an edge table of EHCAP entries per
// workgroup from the global slab `eslab` (EHCAP 0: pairwise scans)
template <int NT, int TIER, int MAXRT, int HCAP, int RFHCAP, int MAXRF, int MAXBE, int QHCAP, int MAXQ,
          int MAXBF, int EHCAP>
QMD void d_grow_lds(Mesh M, int cls, Cands C, Pools PL, BfPool BP, const int* list, int nlist, char* eslab,
                    int min_tier, const int bid, const int gdim) {
    __shared__ int rt[MAXRT];
    __shared__ unsigned H[HCAP];
    __shared__ unsigned RFH[RFHCAP];
    __shared__ int rf[MAXRF];
    __shared__ int4 be[MAXBE];
    __shared__ unsigned long long QH[QHCAP];
    __shared__ int2 q[MAXQ];
    __shared__ int4 cx4[(CXW * MAXBF + MAXBF + 3) / 4];
    int* cx = reinterpret_cast<int*>(cx4);
    __shared__ GrowShared S;
    GrowTiles W{rt, H, RFH, rf, be, QH, q, cx, MAXRT, HCAP, RFHCAP, MAXRF, MAXBE, QHCAP, MAXQ, MAXBF, MAXBF, TIER,
                nullptr, nullptr, 0};
    if (EHCAP > 0) {
        char* base = eslab + (size_t)bid * EHCAP * (sizeof(unsigned long long) + sizeof(int4));
        W.EK = (unsigned long long*)base;
        W.EV = (int4*)(base + (size_t)EHCAP * sizeof(unsigned long long));
        W.ehcap = EHCAP;
    }
    prof_begin(S);
    // all candidates in priority order, or the re-run list (pool-full ones)
    const int n = list ? nlist : C.n;
    for (int i = bid; i < n; i += gdim) {
        const int cid = list ? list[i] : i;
        if (C.st[cid] != ST_PENDING) {
            if (threadIdx.x == 0) { C.gst[cid] = C.st[cid]; C.greason[cid] = C.reason[cid]; }
            continue;
        }
        if (TIER == 0) {            // start at a larger tier: test option, or the tet's remembered tier
            int start = min_tier;
            if (cls == CLS_TET) {
                const unsigned h = (M.TI[C.elem[cid]] >> TI_HINT_SHIFT) & 3u;
                start = max(start, h == 3u ? 2 : (int)h);
            }
            if (start > 0) {
                if (threadIdx.x == 0) C.gst[cid] = start == 1 ? ST_OVERFLOW : ST_OVERFLOW2;
                continue;
            }
        }
        grow_one<NT>(M, cls, C, PL, BP, cid, W, S);
        __syncthreads();
        tier_count(S, BP, TIER);
    }
    prof_flush(S, BP, TIER);
}
template <int NT, int TIER, int MAXRT, int HCAP, int RFHCAP, int MAXRF, int MAXBE, int QHCAP, int MAXQ,
          int MAXBF, int EHCAP>
__global__ __launch_bounds__(NT) void k_grow_lds(Mesh M, int cls, Cands C, Pools PL, BfPool BP,
                                                 const int* list, int nlist, char* eslab, int min_tier) {
    d_grow_lds<NT, TIER, MAXRT, HCAP, RFHCAP, MAXRF, MAXBE, QHCAP, MAXQ, MAXBF, EHCAP>(
        M, cls, C, PL, BP, list, nlist, eslab, min_tier, blockIdx.x, gridDim.x);
}

// carve the tiles other than the hash tables from a workgroup's slab block
QMD void carve_lists(GrowTiles& W, const GrowTiles& T, char* base) {
    size_t off = 0;
    auto carve = [&](size_t bytes) { char* p = base + off; off += (bytes + 255) & ~(size_t)255; return p; };
    W.rt = (int*)carve(sizeof(int) * T.maxrt);
    W.rf = (int*)carve(sizeof(int) * T.maxrf);
    W.be = (int4*)carve(sizeof(int4) * T.maxbe);
    W.q = (int2*)carve(sizeof(int2) * T.maxq);
    W.cx = (int*)carve(sizeof(int) * (CXW * T.maxbf + T.maxcx));
    W.EK = (unsigned long long*)carve(sizeof(unsigned long long) * T.ehcap);
    W.EV = (int4*)carve(sizeof(int4) * T.ehcap);
}
inline size_t lists_slab_bytes(const GrowTiles& T) {
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return r(sizeof(int) * T.maxrt) + r(sizeof(int) * T.maxrf) + r(sizeof(int4) * T.maxbe) +
           r(sizeof(int2) * T.maxq) + r(sizeof(int) * (CXW * T.maxbf + T.maxcx)) +
           r(sizeof(unsigned long long) * T.ehcap) + r(sizeof(int4) * T.ehcap);
}

// Hybrid tier: the three hash tables (tested tets, facet region, queue: the
// atomic-heavy structures) in LDS, the region list, face records and edge
// table in the workgroup's block of a global slab.  `list` holds the
// candidate ids; T carries the capacities (hcap = HCAP, ...).
// (`block`: this workgroup's block of the slab).  With `next` (a counter
// zeroed before the launch) each workgroup takes the next candidate of the
// list when it is done with one, so that regions of very different sizes even
// out over the workgroups; without it, workgroup bid takes every gdim-th.
template <int NT, int HCAP, int RFHCAP, int QHCAP>
QMD void d_grow_hybrid(Mesh M, int cls, Cands C, Pools PL, BfPool BP, const int* list, int nlist,
                       const GrowTiles& T, char* block, const int bid, const int gdim, int* next = nullptr) {
    __shared__ unsigned H[HCAP];
    __shared__ unsigned RFH[RFHCAP];
    __shared__ unsigned long long QH[QHCAP];
    __shared__ GrowShared S;
    GrowTiles W = T;
    carve_lists(W, T, block);
    W.H = H; W.RFH = RFH; W.QH = QH;
    W.hcap = HCAP; W.rfhcap = RFHCAP; W.qhcap = QHCAP;
    prof_begin(S);
    for (int i = bid;; i += gdim) {
        if (next) {
            if (threadIdx.x == 0) S.take = atomicAdd(next, 1);
            __syncthreads();
            i = S.take;                   // every lane reads it before the barriers of grow_one
        }
        if (i >= nlist) break;
        grow_one<NT>(M, cls, C, PL, BP, list[i], W, S);
        __syncthreads();
        tier_count(S, BP, 1);
    }
    prof_flush(S, BP, 1);
}
template <int NT, int HCAP, int RFHCAP, int QHCAP>
__global__ __launch_bounds__(NT) void k_grow_hybrid(Mesh M, int cls, Cands C, Pools PL, BfPool BP,
                                                    const int* list, int nlist, GrowTiles T, char* slab,
                                                    size_t slab_per_block, int* next) {
    d_grow_hybrid<NT, HCAP, RFHCAP, QHCAP>(M, cls, C, PL, BP, list, nlist, T, slab + slab_per_block * blockIdx.x,
                                           blockIdx.x, gridDim.x, next);
}

// re-run of the candidates that overflowed the LDS tiles (or a pool), with
// tiles carved from a global scratch slab; `list` holds their ids
template <int NT>
QMD void d_grow_global(Mesh M, int cls, Cands C, Pools PL, BfPool BP, const int* list, int nlist,
                       const GrowTiles& T, char* base, const int bid, const int gdim) {
    __shared__ GrowShared S;
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
    W.cx = (int*)carve(sizeof(int) * (CXW * T.maxbf + T.maxcx));
    W.EK = (unsigned long long*)carve(sizeof(unsigned long long) * T.ehcap);
    W.EV = (int4*)carve(sizeof(int4) * T.ehcap);
    prof_begin(S);
    for (int i = bid; i < nlist; i += gdim) {
        grow_one<NT>(M, cls, C, PL, BP, list[i], W, S);
        __syncthreads();
        tier_count(S, BP, 2);
    }
    prof_flush(S, BP, 2);
}
template <int NT>
__global__ __launch_bounds__(NT) void k_grow_global(Mesh M, int cls, Cands C, Pools PL, BfPool BP,
                                                    const int* list, int nlist, GrowTiles T, char* slab,
                                                    size_t slab_per_block) {
    d_grow_global<NT>(M, cls, C, PL, BP, list, nlist, T, slab + slab_per_block * blockIdx.x, blockIdx.x,
                      gridDim.x);
}

inline size_t grow_slab_bytes(const GrowTiles& T) {
    auto r = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return r(sizeof(int) * T.maxrt) + r(sizeof(unsigned) * T.hcap) + r(sizeof(unsigned) * T.rfhcap) +
           r(sizeof(int) * T.maxrf) + r(sizeof(int4) * T.maxbe) + r(sizeof(unsigned long long) * T.qhcap) +
           r(sizeof(int2) * T.maxq) + r(sizeof(int) * (CXW * T.maxbf + T.maxcx)) +
           r(sizeof(unsigned long long) * T.ehcap) + r(sizeof(int4) * T.ehcap);
}

}  // namespace qm
