// qm_setup.h -- device-side setup from the input arrays (adjacency, subface
// and subsegment marks, facet projection axes, h_min) and output compaction.
#pragma once
#include "qm_kernels.h"

namespace qm {

// vertices: pack to double4, check the coordinate lattice and the cube
__global__ void k_setup_verts(int nv, const double* xyz, double4* X, int* err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double x = xyz[3 * (size_t)i], y = xyz[3 * (size_t)i + 1], z = xyz[3 * (size_t)i + 2];
    bool ok = true;
    for (double c : {x, y, z}) {
        if (!(c >= 0.0 && c <= 1.0)) ok = false;
        else if (rint(c * kLat) != c * kLat) ok = false;
    }
    if (!ok) atomicOr(err, 1);
    X[i] = make_double4(x, y, z, 0.0);
}

// tets: copy, check ids and positive orientation; `tfl` (resumed
// refinement, else null): bit0 exempt
__global__ void k_setup_tets(int nt, int nv, const int* tin, const unsigned char* tfl, Mesh M, int* err) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int4 v = make_int4(tin[4 * (size_t)t], tin[4 * (size_t)t + 1], tin[4 * (size_t)t + 2], tin[4 * (size_t)t + 3]);
    if (v.x < 0 || v.y < 0 || v.z < 0 || v.w < 0 || v.x >= nv || v.y >= nv || v.z >= nv || v.w >= nv) {
        atomicOr(err, 1);
        v = make_int4(0, 0, 0, 0);
    } else {
        double A[3], B[3], Cc[3], D[3];
        xyz(M, v.x, A); xyz(M, v.y, B); xyz(M, v.z, Cc); xyz(M, v.w, D);
        if (orient3d_any(A, B, Cc, D, M.err) <= 0) atomicOr(err, 2);
    }
    *reinterpret_cast<int4*>(M.TV + 4 * (size_t)t) = v;
    M.TI[t] = TI_ALIVE | (tfl && (tfl[t] & 1u) ? (unsigned)TI_EXEMPT : 0u);
}

QMD unsigned long long face_key3(int a, int b, int c) {
    sort3(a, b, c);
    return ((unsigned long long)a << 42) | ((unsigned long long)b << 21) | (unsigned long long)c;
}
__global__ void k_face_keys(int nt, const int* TV, unsigned long long* keys, int* vals) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * nt) return;
    int t = i >> 2, f = i & 3;
    int4 v = ld4(TV, t);
    keys[i] = face_key3(at4(v, c_FI[f][0]), at4(v, c_FI[f][1]), at4(v, c_FI[f][2]));
    vals[i] = i;
}
__global__ void k_face_match(int n, const unsigned long long* k, const int* v, int* TA, int* err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool prev = i > 0 && k[i - 1] == k[i], next = i + 1 < n && k[i + 1] == k[i];
    if (prev && next) { atomicOr(err, 4); return; }
    if (next) { TA[v[i]] = v[i + 1]; TA[v[i + 1]] = v[i]; }
    else if (!prev) TA[v[i]] = -1;
}
QMD int lower_bound64(const unsigned long long* k, int n, unsigned long long key) {
    int lo = 0, hi = n;
    while (lo < hi) { int mid = (lo + hi) >> 1; if (k[mid] < key) lo = mid + 1; else hi = mid; }
    return lo;
}
// `sfl` (resumed refinement, else null): bit0 queued, bit1 exempt, set on
// both tets of the subface as the rounds set them
__global__ void k_mark_subfaces(int nsf, int nv, int nfacet, const int* sf, const int* sff,
                                const unsigned char* sfl, const unsigned long long* k, const int* v, int n,
                                int* TF, unsigned* TI, int* err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsf) return;
    int a = sf[3 * (size_t)i], b = sf[3 * (size_t)i + 1], c = sf[3 * (size_t)i + 2], F = sff[i];
    if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv || F < 0 || F >= nfacet) { atomicOr(err, 1); return; }
    unsigned long long key = face_key3(a, b, c);
    int j = lower_bound64(k, n, key);
    if (j >= n || k[j] != key) { atomicOr(err, 8); return; }
    const unsigned fl = sfl ? sfl[i] : 0u;
    for (; j < n && k[j] == key; ++j) {
        const int f = v[j] & 3;
        TF[v[j]] = F;
        atomicOr(&TI[v[j] >> 2], ti_fsub(f) | ((fl & 1u) << (4 + f)) | (((fl >> 1) & 1u) << (8 + f)));
    }
}
__global__ void k_edge_keys(int nt, const int* TV, unsigned long long* keys, int* vals) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * nt) return;
    int t = i / 6, e = i % 6;
    int4 v = ld4(TV, t);
    int a = at4(v, c_EV[e][0]), b = at4(v, c_EV[e][1]);
    if (b < a) { int x = a; a = b; b = x; }
    keys[i] = ((unsigned long long)a << 32) | (unsigned)b;
    vals[i] = i;
}
// `ssl` (resumed refinement, else null): bit0 queued, bit1 exempt
__global__ void k_mark_subsegs(int nss, int nv, const int* ss, const int* ssg, const unsigned char* ssl,
                               const unsigned long long* k, const int* v, int n, Mesh M, int* err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nss) return;
    int a = ss[2 * (size_t)i], b = ss[2 * (size_t)i + 1];
    if (a < 0 || b < 0 || a >= nv || b >= nv || a == b) { atomicOr(err, 1); return; }
    if (b < a) { int x = a; a = b; b = x; }
    unsigned long long key = ((unsigned long long)a << 32) | (unsigned)b;
    int j = lower_bound64(k, n, key);
    if (j >= n || k[j] != key) { atomicOr(err, 16); return; }
    M.STET[i] = v[j] / 6;
    for (; j < n && k[j] == key; ++j) M.TS[v[j]] = i;
    M.SV[i] = make_int2(a, b); M.SSEG[i] = ssg[i]; M.SFL[i] = ssl ? (ssl[i] & 3u) : 0u;
}
// projection axis of each facet: the dominant normal component of the
// 1 + the largest id of ids[0..n) into *out (atomic max; *out starts at 0)
__global__ void k_count_ids(int n, const int* ids, int* out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(out, ids[i] + 1);
}
// facet's first PLC triangle (lowest index), ties to the lower axis
__global__ void k_facet_first(int nftri, const int* ff, int nfacet, int* first, int* err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nftri) return;
    int F = ff[i];
    if (F < 0 || F >= nfacet) { atomicOr(err, 1); return; }
    atomicMin(&first[F], i);
}
__global__ void k_facet_axis(int nfacet, const int* first, const int* ftri, const double4* X, int nv, int* FAX,
                             int* err) {
    int F = blockIdx.x * blockDim.x + threadIdx.x;
    if (F >= nfacet) return;
    int i = first[F];
    if (i == 0x7fffffff) { FAX[F] = 2; return; }             // facet with no triangle: unused
    int ia = ftri[3 * (size_t)i], ib = ftri[3 * (size_t)i + 1], ic = ftri[3 * (size_t)i + 2];
    if (ia < 0 || ib < 0 || ic < 0 || ia >= nv || ib >= nv || ic >= nv) { atomicOr(err, 1); return; }
    double4 a = X[ia], b = X[ib], c = X[ic];
    double u0 = b.x - a.x, u1 = b.y - a.y, u2 = b.z - a.z;
    double w0 = c.x - a.x, w1 = c.y - a.y, w2 = c.z - a.z;
    double n0 = fabs(u1 * w2 - u2 * w1), n1 = fabs(u2 * w0 - u0 * w2), n2 = fabs(u0 * w1 - u1 * w0);
    int ax = 0;
    if (n1 > n0) ax = 1;
    if (n2 > (ax == 0 ? n0 : n1)) ax = 2;
    FAX[F] = ax;
}
// shortest squared edge of the input (for h_min); non-negative doubles order
// like their bit patterns
__global__ void k_min_edge(int nt, Mesh M, unsigned long long* out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int4 v = ld4(M.TV, t);
    double P[4][3];
    for (int i = 0; i < 4; ++i) xyz(M, at4(v, i), P[i]);
    double m = INFINITY;
    for (int e = 0; e < 6; ++e) { double d = d2(P[c_EV[e][0]], P[c_EV[e][1]]); if (d < m) m = d; }
    atomicMin(out, (unsigned long long)__double_as_longlong(m));
}

// ------------------------------------------------------------------ slot order
// Tets are renumbered now and then in Morton order of their centroids, so
// that tets near each other in space sit near each other in memory and one
// cache line serves several gathers of a region.  Slots never decide a
// result, so the order is free.
QMD unsigned spread3(unsigned x) {      // 10 bits -> every third of 30 bits
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}
__global__ void k_order_keys(Mesh M, unsigned long long* key, int* val, int* nalive) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M.nt) return;
    val[t] = t;
    if (!(M.TI[t] & TI_ALIVE)) { key[t] = 0xFFFFFFFF00000000ull | (unsigned)t; return; }
    atomicAdd(nalive, 1);
    const int4 v = ld4(M.TV, t);
    const double4 a = M.X[v.x], b = M.X[v.y], c = M.X[v.z], d = M.X[v.w];
    auto q = [](double s) { int k = (int)(s * 256.0); return (unsigned)(k < 0 ? 0 : (k > 1023 ? 1023 : k)); };
    const unsigned m = spread3(q(a.x + b.x + c.x + d.x)) | (spread3(q(a.y + b.y + c.y + d.y)) << 1) |
                       (spread3(q(a.z + b.z + c.z + d.z)) << 2);
    key[t] = ((unsigned long long)m << 32) | (unsigned)t;
}
// new slot of every old slot (dead ones land after the live ones)
__global__ void k_order_perm(int nt, const int* order, int* perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nt) perm[order[i]] = i;
}
// live tets gathered into their new slots, neighbour links renumbered
__global__ void k_order_gather(int nlive, const int* order, const int* perm, Mesh M, int* TV, int* TA, int* TF,
                               int* TS, unsigned* TI) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nlive) return;
    const int t = order[i];
    *reinterpret_cast<int4*>(TV + 4 * (size_t)i) = ld4(M.TV, t);
    *reinterpret_cast<int4*>(TF + 4 * (size_t)i) = ld4(M.TF, t);
    int4 a = ld4(M.TA, t);
    auto re = [&](int nb) { return nb < 0 ? -1 : (perm[nb >> 2] << 2) | (nb & 3); };
    *reinterpret_cast<int4*>(TA + 4 * (size_t)i) = make_int4(re(a.x), re(a.y), re(a.z), re(a.w));
    for (int e = 0; e < 6; ++e) TS[6 * (size_t)i + e] = M.TS[6 * (size_t)t + e];
    TI[i] = M.TI[t];
}
__global__ void k_order_stet(int nss, const int* perm, int* STET) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nss) STET[s] = perm[STET[s]];
}

// ------------------------------------------------------------------ output
__global__ void k_out_flags(Mesh M, int* tflag, int* sfflag) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M.nt) return;
    bool alive = (M.TI[t] & TI_ALIVE) != 0;
    tflag[t] = alive;
    int4 v = ld4(M.TV, t);
    for (int f = 0; f < 4; ++f) {
        int keep = 0;
        if (alive && M.TF[4 * (size_t)t + f] >= 0) {
            int nb = M.TA[4 * (size_t)t + f];
            keep = nb < 0 || at4(v, f) < M.TV[4 * (size_t)(nb >> 2) + (nb & 3)];
        }
        sfflag[4 * (size_t)t + f] = keep;
    }
}
__global__ void k_out_tets(Mesh M, const int* tflag, const int* tscan, int* out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M.nt || !tflag[t]) return;
    *reinterpret_cast<int4*>(out + 4 * (size_t)tscan[t]) = ld4(M.TV, t);
}
__global__ void k_out_sf(Mesh M, const int* flag, const int* scan, int* sf, int* sff) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * M.nt || !flag[i]) return;
    int t = i >> 2, f = i & 3;
    int4 v = ld4(M.TV, t);
    int a = at4(v, c_FI[f][0]), b = at4(v, c_FI[f][1]), c = at4(v, c_FI[f][2]);
    sort3(a, b, c);
    int o = scan[i];
    sf[3 * (size_t)o] = a; sf[3 * (size_t)o + 1] = b; sf[3 * (size_t)o + 2] = c;
    sff[o] = M.TF[i];
}
// the refinement state of the output, aligned with k_out_tets and k_out_sf:
// a tet's exempt bit, a subface's queued and exempt bits (from the tet that
// holds its output copy, the one classification reads) and a subsegment's
__global__ void k_out_state(Mesh M, const int* tflag, const int* tscan, const int* sfflag, const int* sfscan,
                            unsigned char* tfl, unsigned char* sfl, unsigned char* ssl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < M.nss) ssl[t] = (unsigned char)(M.SFL[t] & 3u);
    if (t >= M.nt || !tflag[t]) return;
    const unsigned ti = M.TI[t];
    tfl[tscan[t]] = (ti & TI_EXEMPT) ? 1 : 0;
    for (int f = 0; f < 4; ++f)
        if (sfflag[4 * (size_t)t + f])
            sfl[sfscan[4 * (size_t)t + f]] = (unsigned char)(((ti >> (4 + f)) & 1u) | (((ti >> (8 + f)) & 1u) << 1));
}
__global__ void k_out_xyz(int nv, const double4* X, double* xyz) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double4 q = X[i];
    xyz[3 * (size_t)i] = q.x; xyz[3 * (size_t)i + 1] = q.y; xyz[3 * (size_t)i + 2] = q.z;
}

}  // namespace qm
