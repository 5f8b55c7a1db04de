// qm_insert.h -- flags, disjoint-set selection and concurrent insertion.
#pragma once
#include "qm_grow.h"

namespace qm {

// final status of each candidate: the walk's verdict if it decided, else the
// region evaluation's
QMD int final_status(const Cands& C, int i) { return C.st[i] != ST_PENDING ? C.st[i] : C.gst[i]; }

// Verdicts of the round, one thread per candidate: rejected points queue
// their targets and exempted elements are marked (before insertion, so a
// flagged element destroyed this round loses its flags with it and new
// elements start clean); the round statistics [ncand, ok, rejected, exempt,
// exempt by reason 1..9, unresolved] are counted per block in LDS; accepted
// candidates enter the selection undecided (state 0), the others never do
// (state 3).
QMD void d_verdicts(Mesh M, int cls, Cands C, Pools PL, int* stats, const int bid, const int gdim) {
    __shared__ int bs[16];
    if (threadIdx.x < 16) bs[threadIdx.x] = 0;
    __syncthreads();
    const int i = bid * blockDim.x + threadIdx.x;
    if (i < C.n) {
        const int st = C.st[i] != ST_PENDING ? C.st[i] : C.gst[i];
        auto queue = [&](int2 e) {
            if (e.x == 0) atomicOr(&M.SFL[e.y], SS_QUEUED);
            else {
                int t = e.y >> 2, f = e.y & 3;
                atomicOr(&M.TI[t], 1u << (4 + f));
                int nb = M.TA[4 * (size_t)t + f];
                if (nb >= 0) atomicOr(&M.TI[nb >> 2], 1u << (4 + (nb & 3)));
            }
        };
        atomicAdd(&bs[0], 1);
        if (st == ST_OK) atomicAdd(&bs[1], 1);
        else if (st == ST_REJECT) {
            atomicAdd(&bs[2], 1);
            if (C.st[i] == ST_REJECT) queue(C.qw[i]);
            else for (int k = 0; k < C.q_n[i]; ++k) queue(PL.q[C.q_off[i] + k]);
        } else if (st == ST_EXEMPT) {
            atomicAdd(&bs[3], 1);
            int r = C.st[i] != ST_PENDING ? C.reason[i] : C.greason[i];
            atomicAdd(&bs[3 + r], 1);
            int e = C.elem[i];
            if (cls == CLS_SS) atomicOr(&M.SFL[e], SS_EXEMPT);
            else if (cls == CLS_SF) {
                int t = e >> 2, f = e & 3;
                atomicOr(&M.TI[t], 1u << (8 + f));
                int nb = M.TA[4 * (size_t)t + f];
                if (nb >= 0) atomicOr(&M.TI[nb >> 2], 1u << (8 + (nb & 3)));
            } else atomicOr(&M.TI[e], TI_EXEMPT);
        } else if (st == ST_LOST) atomicAdd(&bs[14], 1);   // stopped early: evaluated again later
        else atomicAdd(&bs[13], 1);     // unresolved (internal error)
        C.state[i] = st == ST_OK ? 0 : 3;
    }
    __syncthreads();
    if (threadIdx.x < 16 && bs[threadIdx.x]) atomicAdd(&stats[threadIdx.x], bs[threadIdx.x]);
}
__global__ __launch_bounds__(256) void k_verdicts(Mesh M, int cls, Cands C, Pools PL, int* stats) {
    d_verdicts(M, cls, C, PL, stats, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------- selection
// Iterated local maxima with fixed priorities: in each pass every undecided
// candidate marks its claim set with its priority (atomic max, skipped when
// the mark already read is as high: marks only grow, and the pass number in
// their high bits makes every earlier mark lower); a candidate
// owning all its marks is kept, one touching a kept claim is dropped.  The
// result is exactly the greedy maximal disjoint set in priority order.
// Passes are launched in batches without waiting: every kernel of a pass
// returns at once when the previous pass left nothing undecided (`prev`).
QMD unsigned long long mis_val(unsigned pass, int c) {
    return ((unsigned long long)pass << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)c);
}
QMD void d_mis_mark(int ncl, const int* cl, const int* clc, const int* state,
                           unsigned long long* mark, unsigned pass, const int* prev, const int bid, const int gdim) {
    int e = bid * blockDim.x + threadIdx.x;
    if (e >= ncl || (prev && *prev == 0)) return;
    int c = clc[e];
    if (c < 0) return;                 // void range (reservation that did not fit)
    if (state[c] != 0) return;
    const unsigned long long v = mis_val(pass, c);
    unsigned long long* const p = &mark[cl[e]];
    if (*p < v) atomicMax(p, v);       // marks only grow: one as high already leaves the atomic nothing to do
}
__global__ void k_mis_mark(int ncl, const int* cl, const int* clc, const int* state,
                           unsigned long long* mark, unsigned pass, const int* prev) {
    d_mis_mark(ncl, cl, clc, state, mark, pass, prev, blockIdx.x, gridDim.x);
}
// per claim entry of an undecided candidate: touching a kept claim drops it
// (drop[c]), a tet marked by a higher priority leaves it undecided (lose[c]);
// every writer stores the same value, so plain stores suffice
QMD void d_mis_check(int ncl, const int* cl, const int* clc, const int* state,
                            const unsigned long long* mark, const int* owner, unsigned pass,
                            unsigned char* drop, unsigned char* lose, const int* prev, const int bid, const int gdim) {
    int e = bid * blockDim.x + threadIdx.x;
    if (e >= ncl || (prev && *prev == 0)) return;
    int c = clc[e];
    if (c < 0 || state[c] != 0) return;
    int t = cl[e];
    if (owner[t] >= 0) drop[c] = 1;
    else if (mark[t] != mis_val(pass, c)) lose[c] = 1;
}
__global__ void k_mis_check(int ncl, const int* cl, const int* clc, const int* state,
                            const unsigned long long* mark, const int* owner, unsigned pass,
                            unsigned char* drop, unsigned char* lose, const int* prev) {
    d_mis_check(ncl, cl, clc, state, mark, owner, pass, drop, lose, prev, blockIdx.x, gridDim.x);
}
// (the first pass of a round; the candidates left undecided are appended
// to the list u_out for the later passes)
QMD void d_mis_decide(int n, int* state, unsigned char* drop, unsigned char* lose,
                                                    int* undecided, const int* prev, int* u_out, int* nu_out, const int bid, const int gdim) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int c = bid * blockDim.x + threadIdx.x;
    if (c < n && !(prev && *prev == 0) && state[c] == 0) {
        if (drop[c]) state[c] = 2;
        else if (lose[c]) { atomicAdd(&cnt, 1); u_out[atomicAdd(nu_out, 1)] = c; }
        else state[c] = 1;
        drop[c] = 0; lose[c] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(undecided, cnt);
}
__global__ __launch_bounds__(256) void k_mis_decide(int n, int* state, unsigned char* drop, unsigned char* lose,
                                                    int* undecided, const int* prev, int* u_out, int* nu_out) {
    d_mis_decide(n, state, drop, lose, undecided, prev, u_out, nu_out, blockIdx.x, gridDim.x);
}

// Passes after the first: only the candidates still undecided take part
// (list u_in, count *nu_in, in any order: every step is order-free).  One
// wave per listed candidate walks its claim range; the decision appends the
// still-undecided ones to u_out.  The mark kernel clears *nu_out (read
// again only by the decision kernel of the same pass).
constexpr int MIS_LIST_GRID = 2048;
QMD void d_mis_mark_list(const int* u_in, const int* nu_in, Cands C, const int* cl,
                                                       unsigned long long* mark, unsigned pass, int* nu_out, const int bid, const int gdim) {
    if (bid == 0 && threadIdx.x == 0) *nu_out = 0;
    const int lane = threadIdx.x & 63, n = *nu_in;
    for (int i = bid * 4 + (threadIdx.x >> 6); i < n; i += gdim * 4) {
        const int c = u_in[i], off = C.cl_off[c], m = C.cl_n[c];
        const unsigned long long v = mis_val(pass, c);
        for (int j = lane; j < m; j += 64) {
            unsigned long long* const p = &mark[cl[off + j]];
            if (*p < v) atomicMax(p, v);
        }
    }
}
__global__ __launch_bounds__(256) void k_mis_mark_list(const int* u_in, const int* nu_in, Cands C, const int* cl,
                                                       unsigned long long* mark, unsigned pass, int* nu_out) {
    d_mis_mark_list(u_in, nu_in, C, cl, mark, pass, nu_out, blockIdx.x, gridDim.x);
}
QMD void d_mis_check_list(const int* u_in, const int* nu_in, Cands C, const int* cl,
                                                        const unsigned long long* mark, const int* owner,
                                                        unsigned pass, unsigned char* drop, unsigned char* lose, const int bid, const int gdim) {
    const int lane = threadIdx.x & 63, n = *nu_in;
    for (int i = bid * 4 + (threadIdx.x >> 6); i < n; i += gdim * 4) {
        const int c = u_in[i], off = C.cl_off[c], m = C.cl_n[c];
        const unsigned long long v = mis_val(pass, c);
        for (int j = lane; j < m; j += 64) {
            const int t = cl[off + j];
            if (owner[t] >= 0) drop[c] = 1;
            else if (mark[t] != v) lose[c] = 1;
        }
    }
}
__global__ __launch_bounds__(256) void k_mis_check_list(const int* u_in, const int* nu_in, Cands C, const int* cl,
                                                        const unsigned long long* mark, const int* owner,
                                                        unsigned pass, unsigned char* drop, unsigned char* lose) {
    d_mis_check_list(u_in, nu_in, C, cl, mark, owner, pass, drop, lose, blockIdx.x, gridDim.x);
}
QMD void d_mis_decide_list(const int* u_in, const int* nu_in, int* state,
                                                         unsigned char* drop, unsigned char* lose, int* undecided,
                                                         int* u_out, int* nu_out, const int bid, const int gdim) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int n = *nu_in;
    for (int i = bid * blockDim.x + threadIdx.x; i < n; i += gdim * blockDim.x) {
        const int c = u_in[i];
        if (drop[c]) state[c] = 2;
        else if (lose[c]) { atomicAdd(&cnt, 1); u_out[atomicAdd(nu_out, 1)] = c; }
        else state[c] = 1;
        drop[c] = 0; lose[c] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(undecided, cnt);
}
__global__ __launch_bounds__(256) void k_mis_decide_list(const int* u_in, const int* nu_in, int* state,
                                                         unsigned char* drop, unsigned char* lose, int* undecided,
                                                         int* u_out, int* nu_out) {
    d_mis_decide_list(u_in, nu_in, state, drop, lose, undecided, u_out, nu_out, blockIdx.x, gridDim.x);
}
QMD void d_mis_commit_list(const int* u_in, const int* nu_in, Cands C, const int* cl,
                                                         const int* state, int* owner, const int bid, const int gdim) {
    const int lane = threadIdx.x & 63, n = *nu_in;
    for (int i = bid * 4 + (threadIdx.x >> 6); i < n; i += gdim * 4) {
        const int c = u_in[i];
        if (state[c] != 1) continue;
        const int off = C.cl_off[c], m = C.cl_n[c];
        for (int j = lane; j < m; j += 64) owner[cl[off + j]] = c;
    }
}
__global__ __launch_bounds__(256) void k_mis_commit_list(const int* u_in, const int* nu_in, Cands C, const int* cl,
                                                         const int* state, int* owner) {
    d_mis_commit_list(u_in, nu_in, C, cl, state, owner, blockIdx.x, gridDim.x);
}
QMD void d_mis_commit(int ncl, const int* cl, const int* clc, const int* state, int* owner,
                             const int* prev, const int bid, const int gdim) {
    int e = bid * blockDim.x + threadIdx.x;
    if (e >= ncl || (prev && *prev == 0)) return;
    int c = clc[e];
    if (c < 0) return;
    if (state[c] == 1) owner[cl[e]] = c;
}
__global__ void k_mis_commit(int ncl, const int* cl, const int* clc, const int* state, int* owner,
                             const int* prev) {
    d_mis_commit(ncl, cl, clc, state, owner, prev, blockIdx.x, gridDim.x);
}
// All passes of a small round in one workgroup (phases separated by block
// barriers): one launch instead of four per pass.  *npass receives the
// passes run, or -1 when max_pass passes did not finish.
QMD void d_mis_small(int ncl, const int* cl, const int* clc, int n, int* state,
                                                    unsigned long long* mark, int* owner, unsigned char* drop,
                                                    unsigned char* lose, unsigned pass0, int max_pass, int* npass, const int bid, const int gdim) {
    __shared__ int undecided;
    for (int k = 0; k < max_pass; ++k) {
        const unsigned pass = pass0 + (unsigned)k;
        for (int e = threadIdx.x; e < ncl; e += blockDim.x) {          // mark
            int c = clc[e];
            if (c >= 0 && state[c] == 0) {
                const unsigned long long v = mis_val(pass, c);
                unsigned long long* const p = &mark[cl[e]];
                if (*p < v) atomicMax(p, v);
            }
        }
        if (threadIdx.x == 0) undecided = 0;
        __syncthreads();
        for (int e = threadIdx.x; e < ncl; e += blockDim.x) {          // check
            int c = clc[e];
            if (c < 0 || state[c] != 0) continue;
            int t = cl[e];
            if (owner[t] >= 0) drop[c] = 1;
            else if (mark[t] != mis_val(pass, c)) lose[c] = 1;
        }
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += blockDim.x) {            // decide
            if (state[c] != 0) continue;
            if (drop[c]) state[c] = 2;
            else if (lose[c]) atomicAdd(&undecided, 1);
            else state[c] = 1;
            drop[c] = 0; lose[c] = 0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < ncl; e += blockDim.x) {          // commit
            int c = clc[e];
            if (c >= 0 && state[c] == 1) owner[cl[e]] = c;
        }
        __syncthreads();
        if (undecided == 0) {
            if (threadIdx.x == 0) *npass = k + 1;
            return;
        }
        __syncthreads();                     // all have read `undecided` before the next reset
    }
    if (threadIdx.x == 0) *npass = -1;
}
__global__ __launch_bounds__(1024) void k_mis_small(int ncl, const int* cl, const int* clc, int n, int* state,
                                                    unsigned long long* mark, int* owner, unsigned char* drop,
                                                    unsigned char* lose, unsigned pass0, int max_pass, int* npass) {
    d_mis_small(ncl, cl, clc, n, state, mark, owner, drop, lose, pass0, max_pass, npass, blockIdx.x, gridDim.x);
}

// clear every ownership of this round (kept candidates, and kept ones that
// a per-round cap demoted afterwards)
QMD void d_mis_release(int ncl, const int* cl, const int* clc, int* owner, const int bid, const int gdim) {
    int e = bid * blockDim.x + threadIdx.x;
    if (e >= ncl || clc[e] < 0) return;
    if (owner[cl[e]] == clc[e]) owner[cl[e]] = -1;
}
__global__ void k_mis_release(int ncl, const int* cl, const int* clc, int* owner) {
    d_mis_release(ncl, cl, clc, owner, blockIdx.x, gridDim.x);
}

// per-candidate values to scan: kept flag, new tet slots (f - k), new
// subsegment slots
__global__ void k_scan_vals(Cands C, int cls, int* vk, int* vt, int* vs) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C.n) return;
    bool kept = C.state[c] == 1;
    vk[c] = kept;
    int d = kept ? C.bf_n[c] - C.reg_n[c] : 0;
    vt[c] = d > 0 ? d : 0;
    vs[c] = kept && cls == CLS_SS;
}
// the three per-candidate values (kept, new tets, new subsegments)
QMD int3 scan_vals(const Cands& C, int cls, int c) {
    bool kept = C.state[c] == 1;
    int d = kept ? C.bf_n[c] - C.reg_n[c] : 0;
    return make_int3(kept ? 1 : 0, d > 0 ? d : 0, kept && cls == CLS_SS ? 1 : 0);
}
// Exclusive scans of the three values and their totals in one workgroup
// (rounds with few candidates: one launch instead of a device-wide scan per
// value).  sk/st/ss as from k_scan_vals + exclusive sums; tot = k_totals.
QMD void d_scan_small(Cands C, int cls, int n, int* sk, int* st, int* ss,
                                                     int* tot, const int bid, const int gdim) {
    __shared__ int3 wsum[16];
    __shared__ int3 carry;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = make_int3(0, 0, 0);
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int c = base + threadIdx.x;
        int3 v = c < n ? scan_vals(C, cls, c) : make_int3(0, 0, 0);
        int3 x = v;                                   // inclusive scan within the wave
        for (int off = 1; off < 64; off <<= 1) {
            int a = __shfl_up(x.x, off, 64), b = __shfl_up(x.y, off, 64), d = __shfl_up(x.z, off, 64);
            if (lane >= off) { x.x += a; x.y += b; x.z += d; }
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int3 pre = carry;                             // waves before this one, chunks before this one
        for (int w = 0; w < wid; ++w) { pre.x += wsum[w].x; pre.y += wsum[w].y; pre.z += wsum[w].z; }
        if (c < n) {
            sk[c] = pre.x + x.x - v.x;
            st[c] = pre.y + x.y - v.y;
            ss[c] = pre.z + x.z - v.z;
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int w = 0; w < 16; ++w) { carry.x += wsum[w].x; carry.y += wsum[w].y; carry.z += wsum[w].z; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { tot[0] = carry.x; tot[1] = carry.y; tot[2] = carry.z; }
}
__global__ __launch_bounds__(1024) void k_scan_small(Cands C, int cls, int n, int* sk, int* st, int* ss,
                                                     int* tot) {
    d_scan_small(C, cls, n, sk, st, ss, tot, blockIdx.x, gridDim.x);
}

// optional cap on insertions per round: only the first `cap` kept survive
__global__ void k_cap_kept(Cands C, const int* sk, int cap) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C.n) return;
    if (C.state[c] == 1 && sk[c] >= cap) C.state[c] = 2;
}
QMD void d_kept_list(Cands C, const int* sk, int* list, const int bid, const int gdim) {
    int c = bid * blockDim.x + threadIdx.x;
    if (c >= C.n) return;
    if (C.state[c] == 1) list[sk[c]] = c;
}
__global__ void k_kept_list(Cands C, const int* sk, int* list) {
    d_kept_list(C, sk, list, blockIdx.x, gridDim.x);
}
__global__ void k_totals(int n, const int* a, const int* av, const int* b, const int* bv, const int* d,
                         const int* dv, int* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = n ? a[n - 1] + av[n - 1] : 0;
        out[1] = n ? b[n - 1] + bv[n - 1] : 0;
        out[2] = n ? d[n - 1] + dv[n - 1] : 0;
    }
}

// ------------------------------------------------------------- insertion
// One workgroup per kept point: the new tets join p to the boundary faces
// (slots of the deleted region tets are reused first, then fresh slots);
// faces through p are linked by matching boundary edges, the outer face to
// the old neighbour (whose back link is patched), subfaces (p, e) are created
// on 2D boundary edges, and a split subsegment becomes (a,p) + (p,b).
QMD void d_insert(Mesh M, int cls, Cands C, Pools PL, BfPool BP,
                                               const int* kept, int nkept, const int* sk, const int* st_,
                                               const int* ss_, int nv0, int nt0, int nss0, int* dead, const int bid, const int gdim) {
    for (int kk = bid; kk < nkept; kk += gdim) {
        const int c = kept[kk];
        const int lane = threadIdx.x;
        const int pid = nv0 + sk[c];
        const int nf = C.bf_n[c], nk = C.reg_n[c];
        const int bf0 = C.bf_off[c], rg0 = C.reg_off[c], be0 = C.be_off[c], nbe = C.be_n[c];
        const int tbase = nt0 + st_[c];
        int sa = -1, sb = -1, s_old = -1, s_new = -1;
        if (cls == CLS_SS) {
            int4 tp = C.tup[c];
            sa = tp.x; sb = tp.y; s_old = C.elem[c]; s_new = nss0 + ss_[c];
        }
        // phase A: read the face flags of the old boundary faces before any
        // slot of this region is overwritten
        for (int j = lane; j < nf; j += 64) {
            int4* rec = BP.r + BFR * (size_t)(bf0 + j);
            int h = rec[2].y;
            unsigned ti = M.TI[h >> 2];
            int f = h & 3;
            rec[1].y = (int)(((ti >> (4 + f)) & 1u) | (((ti >> (8 + f)) & 1u) << 1));
        }
        __syncthreads();
        auto slot = [&](int j) { return j < nk ? PL.cl[rg0 + j] : tbase + (j - nk); };
        // phase B: write the new tets
        for (int j = lane; j < nf; j += 64) {
            const int4* rec = BP.r + BFR * (size_t)(bf0 + j);
            const int4 r0 = rec[0], r1 = rec[1], r2 = rec[2], r3 = rec[3];
            const int x = r0.x, y = r0.y, z = r0.z;
            const int sj = slot(j);
            // faces through p: opposite x holds edge (y,z), opposite y (x,z),
            // opposite z (x,y); the neighbour across each is the new tet of the
            // boundary face sharing that edge (recorded by the validation)
            const int ea[3] = {y, x, x}, eb[3] = {z, z, y};
            const int pr[3] = {r3.x, r3.y, r3.z};
            int adj[3], fid[3];
            for (int l = 0; l < 3; ++l) {
                adj[l] = pr[l] < 0 ? -1 : ((slot(pr[l] >> 2) << 2) | (pr[l] & 3));
                fid[l] = -1;
                const int u = ea[l], w = eb[l];
                const int lo = u < w ? u : w, hi = u < w ? w : u;
                for (int m = 0; m < nbe; ++m) {
                    int4 e = PL.be[be0 + m];
                    if (e.x == lo && e.y == hi) { fid[l] = e.z; break; }
                }
            }
            *reinterpret_cast<int4*>(M.TV + 4 * (size_t)sj) = make_int4(x, y, z, pid);
            *reinterpret_cast<int4*>(M.TA + 4 * (size_t)sj) = make_int4(adj[0], adj[1], adj[2], r0.w);
            *reinterpret_cast<int4*>(M.TF + 4 * (size_t)sj) = make_int4(fid[0], fid[1], fid[2], r1.x);
            // edges of (x,y,z,p): (0,1)=xy (0,2)=xz (0,3)=xp (1,2)=yz (1,3)=yp (2,3)=zp
            auto sp = [&](int v) { return v == sa ? s_old : (v == sb ? s_new : -1); };
            int* ts = M.TS + 6 * (size_t)sj;
            ts[0] = r1.z; ts[1] = r2.x; ts[2] = sp(x); ts[3] = r1.w; ts[4] = sp(y); ts[5] = sp(z);
            // a fresh info word: no cached classification yet
            M.TI[sj] = TI_ALIVE | ((unsigned)(r1.y & 1) << 7) | ((unsigned)((r1.y >> 1) & 1) << 11) |
                       (fid[0] >= 0 ? ti_fsub(0) : 0u) | (fid[1] >= 0 ? ti_fsub(1) : 0u) |
                       (fid[2] >= 0 ? ti_fsub(2) : 0u) | (r1.x >= 0 ? ti_fsub(3) : 0u);
            if (r0.w >= 0) {
                M.TA[4 * (size_t)(r0.w >> 2) + (r0.w & 3)] = (sj << 2) | 3;
                // the old tet across a boundary subface has a new apex opposite it
                if (r1.x >= 0) atomicAnd(&M.TI[r0.w >> 2], ~ti_fknown(r0.w & 3));
            }
            for (int e = 0; e < 6; ++e) if (ts[e] >= 0) M.STET[ts[e]] = sj;
            // subsegments on the boundary face's edges have new tets in their
            // link (those through p are new or rewritten below)
            for (int e : {0, 1, 3}) if (ts[e] >= 0) atomicAnd(&M.SFL[ts[e]], ~SS_KNOWN);
        }
        for (int j = nf + lane; j < nk; j += 64) M.TI[PL.cl[rg0 + j]] = 0u;   // unused region slots
        if (lane == 0 && nk > nf) atomicAdd(dead, nk - nf);
        if (lane == 0) {
            double4 p = C.p[c];
            M.X[pid] = make_double4(p.x, p.y, p.z, 0.0);
            if (cls == CLS_SS) {
                int seg = M.SSEG[s_old];
                M.SV[s_old] = make_int2(sa, pid); M.SFL[s_old] = 0u;
                M.SV[s_new] = make_int2(sb, pid); M.SFL[s_new] = 0u; M.SSEG[s_new] = seg;
            }
        }
        __syncthreads();
    }
}
__global__ __launch_bounds__(64) void k_insert(Mesh M, int cls, Cands C, Pools PL, BfPool BP,
                                               const int* kept, int nkept, const int* sk, const int* st_,
                                               const int* ss_, int nv0, int nt0, int nss0, int* dead) {
    d_insert(M, cls, C, PL, BP, kept, nkept, sk, st_, ss_, nv0, nt0, nss0, dead, blockIdx.x, gridDim.x);
}

}  // namespace qm
