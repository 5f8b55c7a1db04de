// qm_geom.h -- device geometry for the refinement kernels (gfx950).
//
// Exact predicates: each is an FP64 evaluation with a semi-static error bound
// (error <= c * eps * permanent, Shewchuk 1997, "Adaptive precision
// floating-point arithmetic and fast robust geometric predicates", Sec. 4);
// when the sign is not certain it is computed exactly.
//
// Every vertex of the mesh is a point of the unit cube on the 2^-53 lattice,
// so the predicates of the region growth, validation and classification
// (orient3d, orient2d, insphere, segment and face encroachment) evaluate
// their polynomial in fixed-width integers held in registers (no scratch
// memory).  Only the tet walk of the locate step can aim at a point outside
// the cube; its orientation tests (orient3d_any, orient2d_any) fall back to
// floating-point expansion arithmetic (same paper, Sec. 2: TWO-SUM,
// TWO-PRODUCT via FMA, FAST-EXPANSION-SUM and SCALE-EXPANSION with zero
// elimination).
//
// Constructions (midpoint, circumcentres, radius-edge test) use one fixed
// FP64 operation order with no contraction (-ffp-contract=off) and IEEE
// division, then round onto the 2^-53 lattice; the same formulas written in
// the same order give the same bits on any IEEE-754 machine.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define QMD __device__ __forceinline__
#define QMN __device__ __noinline__

namespace qm {

constexpr double kEps = 1.1102230246251565e-16;   // 2^-53
constexpr double kLat = 9007199254740992.0;       // 2^53
constexpr double kInvLat = 1.0 / 9007199254740992.0;

// Every exact path takes `err`, the calling refinement's own error word: a
// broken precondition (never expected) sets a bit there, and the host reports
// it as an internal error of that call only.

// ------------------------------------------------------------ error-free ops
QMD void two_sum(double a, double b, double& x, double& y) {
    x = a + b;
    double bv = x - a, av = x - bv;
    y = (a - av) + (b - bv);
}
QMD void two_diff(double a, double b, double& x, double& y) {
    x = a - b;
    double bv = a - x, av = x + bv;
    y = (a - av) + (bv - b);
}
QMD void fast_two_sum(double a, double b, double& x, double& y) {   // |a| >= |b|
    x = a + b;
    y = b - (x - a);
}
QMD void two_prod(double a, double b, double& x, double& y) {
    x = a * b;
    y = fma(a, b, -x);
}

// expansions: components in increasing magnitude, zero-eliminated; length 0
// is the value zero.
QMD int exp_diff(double a, double b, double* h) {   // a - b as an expansion
    double x, y;
    two_diff(a, b, x, y);
    int n = 0;
    if (y != 0.0) h[n++] = y;
    if (x != 0.0) h[n++] = x;
    return n;
}

// FAST-EXPANSION-SUM: merge by magnitude, then chain TWO-SUM
__device__ inline int exp_sum(int en, const double* e, int fn, const double* f, double* h) {
    if (en == 0) { for (int i = 0; i < fn; ++i) h[i] = f[i]; return fn; }
    if (fn == 0) { for (int i = 0; i < en; ++i) h[i] = e[i]; return en; }
    int i = 0, j = 0, n = 0;
    double Q;
    if (fabs(e[0]) <= fabs(f[0])) Q = e[i++]; else Q = f[j++];
    while (i < en || j < fn) {
        double g;
        if (j >= fn || (i < en && fabs(e[i]) <= fabs(f[j]))) g = e[i++]; else g = f[j++];
        double s, hh;
        two_sum(Q, g, s, hh);
        if (hh != 0.0) h[n++] = hh;
        Q = s;
    }
    if (Q != 0.0 || n == 0) h[n++] = Q;
    if (n == 1 && h[0] == 0.0) return 0;
    return n;
}

// SCALE-EXPANSION
__device__ inline int exp_scale(int en, const double* e, double b, double* h) {
    if (en == 0 || b == 0.0) return 0;
    double Q, hh;
    int n = 0;
    two_prod(e[0], b, Q, hh);
    if (hh != 0.0) h[n++] = hh;
    for (int i = 1; i < en; ++i) {
        double p1, p0, s;
        two_prod(e[i], b, p1, p0);
        two_sum(Q, p0, s, hh);
        if (hh != 0.0) h[n++] = hh;
        fast_two_sum(p1, s, Q, hh);
        if (hh != 0.0) h[n++] = hh;
    }
    if (Q != 0.0) h[n++] = Q;
    return n;
}

QMD void exp_neg(int n, double* e) { for (int i = 0; i < n; ++i) e[i] = -e[i]; }
QMD int exp_sign(int n, const double* e) { return n == 0 ? 0 : (e[n - 1] > 0.0 ? 1 : (e[n - 1] < 0.0 ? -1 : 0)); }
QMD void exp_copy(int n, const double* s, double* d) { for (int i = 0; i < n; ++i) d[i] = s[i]; }

// product of two expansions: sum over b's components of a scaled copy of a.
// s must hold 2*an, acc and tmp the result bound.
__device__ inline int exp_mul(int an, const double* a, int bn, const double* b, double* out, double* s,
                              double* tmp, int cap, int* err) {
    int n = 0;
    for (int j = 0; j < bn; ++j) {
        int sn = exp_scale(an, a, b[j], s);
        int m = exp_sum(n, out, sn, s, tmp);
        if (m > cap) { atomicOr(err, 1); m = cap; }
        exp_copy(m, tmp, out);
        n = m;
    }
    return n;
}

// --------------------------------------------- predicates on any finite point
// The tet walk of the locate step may aim at a splitting point outside the
// unit cube (a circumcentre far from its tet), so its orientation tests take
// arbitrary finite coordinates: exact fallback in expansion arithmetic.

// sign of det[b-a; c-a; d-a]
QMN int orient3d_any_exact(const double* a, const double* b, const double* c, const double* d, int* err) {
    double u[3][2], v[3][2], w[3][2];
    int un[3], vn[3], wn[3];
    for (int k = 0; k < 3; ++k) {
        un[k] = exp_diff(b[k], a[k], u[k]);
        vn[k] = exp_diff(c[k], a[k], v[k]);
        wn[k] = exp_diff(d[k], a[k], w[k]);
    }
    double acc[192], tmp[256], p1[8], p2[8], mn[16], t[64], s[32];
    int an = 0;
    for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        int n1 = exp_mul(vn[k1], v[k1], wn[k2], w[k2], p1, s, tmp, 8, err);
        int n2 = exp_mul(vn[k2], v[k2], wn[k1], w[k1], p2, s, tmp, 8, err);
        exp_neg(n2, p2);
        int mnn = exp_sum(n1, p1, n2, p2, mn);
        int tn = exp_mul(mnn, mn, un[k], u[k], t, s, tmp, 64, err);
        int m = exp_sum(an, acc, tn, t, tmp);
        exp_copy(m, tmp, acc);
        an = m;
    }
    return exp_sign(an, acc);
}

// FP64 value of det[b-a; c-a; d-a] and its permanent (error scale)
QMD void orient3d_fp(const double* a, const double* b, const double* c, const double* d, double& det,
                     double& per) {
    double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
    double v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
    double w0 = d[0] - a[0], w1 = d[1] - a[1], w2 = d[2] - a[2];
    double m0a = v1 * w2, m0b = v2 * w1, m1a = v2 * w0, m1b = v0 * w2, m2a = v0 * w1, m2b = v1 * w0;
    det = u0 * (m0a - m0b) + u1 * (m1a - m1b) + u2 * (m2a - m2b);
    per = fabs(u0) * (fabs(m0a) + fabs(m0b)) + fabs(u1) * (fabs(m1a) + fabs(m1b))
        + fabs(u2) * (fabs(m2a) + fabs(m2b));
}
constexpr double kO3 = (7.0 + 56.0 * kEps) * kEps;
constexpr double kO2 = (3.0 + 16.0 * kEps) * kEps;

QMD int orient3d_any(const double* a, const double* b, const double* c, const double* d, int* err) {
    double det, per;
    orient3d_fp(a, b, c, d, det, per);
    double bound = kO3 * per;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient3d_any_exact(a, b, c, d, err);
}

// 2D orientation after dropping coordinate `ax` (kept: ax+1, ax+2 mod 3)
QMN int orient2d_any_exact(int ax, const double* a, const double* b, const double* c, int* err) {
    int i = (ax + 1) % 3, j = (ax + 2) % 3;
    double ux[2], uy[2], vx[2], vy[2];
    int uxn = exp_diff(b[i], a[i], ux), uyn = exp_diff(b[j], a[j], uy);
    int vxn = exp_diff(c[i], a[i], vx), vyn = exp_diff(c[j], a[j], vy);
    double p1[8], p2[8], s[4], tmp[16], out[16];
    int n1 = exp_mul(uxn, ux, vyn, vy, p1, s, tmp, 8, err);
    int n2 = exp_mul(uyn, uy, vxn, vx, p2, s, tmp, 8, err);
    exp_neg(n2, p2);
    int n = exp_sum(n1, p1, n2, p2, out);
    return exp_sign(n, out);
}

QMD void orient2d_fp(int ax, const double* a, const double* b, const double* c, double& det, double& per) {
    int i = (ax + 1) % 3, j = (ax + 2) % 3;
    double ux = b[i] - a[i], uy = b[j] - a[j], vx = c[i] - a[i], vy = c[j] - a[j];
    double l = ux * vy, r = uy * vx;
    det = l - r;
    per = fabs(l) + fabs(r);
}

QMD int orient2d_any(int ax, const double* a, const double* b, const double* c, int* err) {
    double det, per;
    orient2d_fp(ax, a, b, c, det, per);
    double bound = kO2 * per;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient2d_any_exact(ax, a, b, c, err);
}

// ------------------------------------------------------- lattice integers
// A point of the unit cube on the 2^-53 lattice is k * 2^-53 with integer
// 0 <= k <= 2^53, so each predicate below is an integer polynomial in the
// k's.  When the FP64 filter cannot decide, the polynomial is evaluated
// exactly in fixed-width two's-complement integers (32-bit limbs, little
// endian, every loop unrolled so the limbs stay in registers).  Widths: a
// form of degree d in coordinate differences (|dk| <= 2^53) with at most m
// terms needs 53 d + log2(m) + 1 bits:
//   orient2d  d = 2   -> 128 bits      segdot   d = 2  -> 128 bits
//   orient3d  d = 3   -> 192 bits      insphere d = 5  -> 288 bits
//   facedot   d = 6   -> 352 bits
template <int N> struct Z { uint32_t w[N]; };

// k = x * 2^53 (exact for lattice points of the cube); off-lattice or
// out-of-cube input is a broken precondition and raises the error flag
QMD int64_t lat(double x, int* err) {
    double k = x * kLat;
    if (!(k >= 0.0 && k <= kLat) || k != rint(k)) atomicOr(err, 256);
    return (int64_t)k;
}
template <int N> QMD Z<N> zfrom(int64_t v) {
    Z<N> r;
    const uint32_t s = v < 0 ? 0xFFFFFFFFu : 0u;
#pragma unroll
    for (int i = 0; i < N; ++i) r.w[i] = i == 0 ? (uint32_t)v : (i == 1 ? (uint32_t)((uint64_t)v >> 32) : s);
    return r;
}
template <int M, int N> QMD Z<M> zext(const Z<N>& a) {   // sign-extend (M >= N)
    Z<M> r;
    const uint32_t s = (int32_t)a.w[N - 1] < 0 ? 0xFFFFFFFFu : 0u;
#pragma unroll
    for (int i = 0; i < M; ++i) r.w[i] = i < N ? a.w[i] : s;
    return r;
}
template <int N> QMD Z<N> zadd(const Z<N>& a, const Z<N>& b) {
    Z<N> r;
    uint64_t c = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint64_t s = (uint64_t)a.w[i] + b.w[i] + c;
        r.w[i] = (uint32_t)s;
        c = s >> 32;
    }
    return r;
}
template <int N> QMD Z<N> zsub(const Z<N>& a, const Z<N>& b) {
    Z<N> r;
    uint64_t br = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint64_t s = (uint64_t)a.w[i] - b.w[i] - br;
        r.w[i] = (uint32_t)s;
        br = s >> 63;
    }
    return r;
}
// -a when neg, else a (two's complement: flip every bit, add one)
template <int N> QMD Z<N> zcneg(const Z<N>& a, bool neg) {
    Z<N> r;
    const uint32_t m = neg ? 0xFFFFFFFFu : 0u;
    uint64_t c = neg ? 1u : 0u;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint64_t s = (uint64_t)(a.w[i] ^ m) + c;
        r.w[i] = (uint32_t)s;
        c = s >> 32;
    }
    return r;
}
// a * b into R limbs (R large enough for the true product): schoolbook on
// the magnitudes, then the sign
template <int R, int A, int B> QMD Z<R> zmul(const Z<A>& a, const Z<B>& b) {
    const bool na = (int32_t)a.w[A - 1] < 0, nb = (int32_t)b.w[B - 1] < 0;
    const Z<A> x = zcneg(a, na);
    const Z<B> y = zcneg(b, nb);
    Z<R> r;
#pragma unroll
    for (int i = 0; i < R; ++i) r.w[i] = 0u;
#pragma unroll
    for (int i = 0; i < A; ++i) {
        uint64_t c = 0;
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (i + j < R) {
                uint64_t t = (uint64_t)x.w[i] * y.w[j] + r.w[i + j] + c;
                r.w[i + j] = (uint32_t)t;
                c = t >> 32;
            }
        }
        if (i + B < R) r.w[i + B] = (uint32_t)c;
    }
    return zcneg(r, na != nb);
}
template <int N> QMD int zsign(const Z<N>& a) {
    if ((int32_t)a.w[N - 1] < 0) return -1;
    uint32_t o = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) o |= a.w[i];
    return o != 0u ? 1 : 0;
}
// difference of two lattice coordinates as a 2-limb integer
QMD Z<2> zd(double x, double y, int* err) { return zfrom<2>(lat(x, err) - lat(y, err)); }
// p*s - q*r for 2-limb operands (|.| <= 2^53): 109 bits
QMD Z<4> zdet2(const Z<2>& p, const Z<2>& q, const Z<2>& r, const Z<2>& s) {
    return zsub(zmul<4>(p, s), zmul<4>(q, r));
}
// dot product of two difference vectors: < 3 * 2^106
QMD Z<4> zdot(const Z<2>* x, const Z<2>* y) {
    return zadd(zadd(zmul<4>(x[0], y[0]), zmul<4>(x[1], y[1])), zmul<4>(x[2], y[2]));
}
// det[u; v; w] of difference vectors: < 2^165
QMD Z<6> zdet3(const Z<2>* u, const Z<2>* v, const Z<2>* w) {
    Z<6> r = zmul<6>(u[0], zdet2(v[1], v[2], w[1], w[2]));
    r = zadd(r, zmul<6>(u[1], zdet2(v[2], v[0], w[2], w[0])));
    return zadd(r, zmul<6>(u[2], zdet2(v[0], v[1], w[0], w[1])));
}

// ------------------------------------- predicates on lattice points of the cube
// orient3d: sign of det[b-a; c-a; d-a]
QMN int orient3d_exact(const double* a, const double* b, const double* c, const double* d, int* err) {
    Z<2> u[3], v[3], w[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) { u[k] = zd(b[k], a[k], err); v[k] = zd(c[k], a[k], err); w[k] = zd(d[k], a[k], err); }
    return zsign(zdet3(u, v, w));
}
QMD int orient3d(const double* a, const double* b, const double* c, const double* d, int* err) {
    double det, per;
    orient3d_fp(a, b, c, d, det, per);
    double bound = kO3 * per;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient3d_exact(a, b, c, d, err);
}

// orient2d in the plane of the coordinates other than `ax`
QMN int orient2d_exact(int ax, const double* a, const double* b, const double* c, int* err) {
    int i = (ax + 1) % 3, j = (ax + 2) % 3;
    return zsign(zdet2(zd(b[i], a[i], err), zd(b[j], a[j], err), zd(c[i], a[i], err), zd(c[j], a[j], err)));
}
QMD int orient2d(int ax, const double* a, const double* b, const double* c, int* err) {
    double det, per;
    orient2d_fp(ax, a, b, c, det, per);
    double bound = kO2 * per;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient2d_exact(ax, a, b, c, err);
}

// insphere: > 0 iff e is strictly inside the circumsphere of positively
// oriented abcd.  With rows r_i = (x_i - e, |x_i - e|^2) the value is
// -det[r_a; r_b; r_c; r_d], expanded along the lifted column.
QMN int insphere_exact(const double* a, const double* b, const double* c, const double* d,
                       const double* e, int* err) {
    const double* r[4] = {a, b, c, d};
    Z<2> m[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) m[i][k] = zd(r[i][k], e[k], err);
    Z<9> acc = zfrom<9>(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r0 = i == 0 ? 1 : 0, r1 = i <= 1 ? 2 : 1, r2 = i <= 2 ? 3 : 2;
        Z<4> lift = zdot(m[i], m[i]);
        Z<9> t = zmul<9>(lift, zdet3(m[r0], m[r1], m[r2]));
        acc = (i & 1) ? zadd(acc, t) : zsub(acc, t);
    }
    return -zsign(acc);
}
QMD int insphere(const double* a, const double* b, const double* c, const double* d, const double* e, int* err) {
    const double* r[4] = {a, b, c, d};
    double m[4][4], pm[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        m[i][0] = r[i][0] - e[0]; m[i][1] = r[i][1] - e[1]; m[i][2] = r[i][2] - e[2];
        m[i][3] = (m[i][0] * m[i][0] + m[i][1] * m[i][1]) + m[i][2] * m[i][2];
#pragma unroll
        for (int k = 0; k < 4; ++k) pm[i][k] = fabs(m[i][k]);
    }
    double det = 0.0, per = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r0 = i == 0 ? 1 : 0, r1 = i <= 1 ? 2 : 1, r2 = i <= 2 ? 3 : 2;
        double d3 = 0.0, p3 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
            d3 += m[r0][k] * (m[r1][k1] * m[r2][k2] - m[r1][k2] * m[r2][k1]);
            p3 += pm[r0][k] * (pm[r1][k1] * pm[r2][k2] + pm[r1][k2] * pm[r2][k1]);
        }
        double t = m[i][3] * d3;
        if ((i + 3) & 1) det -= t; else det += t;
        per += pm[i][3] * p3;
    }
    double bound = (16.0 + 224.0 * kEps) * kEps * per;
    if (-det > bound) return 1;
    if (det > bound) return -1;
    return insphere_exact(a, b, c, d, e, err);
}

// segment encroachment: sign of (v-a).(v-b); negative iff v is strictly
// inside the diametral ball of ab
QMN int segdot_exact(const double* a, const double* b, const double* v, int* err) {
    Z<2> x[3], y[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) { x[k] = zd(v[k], a[k], err); y[k] = zd(v[k], b[k], err); }
    return zsign(zdot(x, y));
}
QMD int segdot(const double* a, const double* b, const double* v, int* err) {
    double val = 0.0, per = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double x = v[k] - a[k], y = v[k] - b[k];
        double t = x * y;
        val += t; per += fabs(t);
    }
    double bound = 8.0 * kEps * per;
    if (val > bound) return 1;
    if (-val > bound) return -1;
    return segdot_exact(a, b, v, err);
}

// face (equatorial ball) encroachment: sign of
//   F = |u x w|^2 |q|^2 - (q.u)|w|^2(|u|^2 - u.w) - (q.w)|u|^2(|w|^2 - u.w),
// u = b-a, w = c-a, q = v-a, with |u x w|^2 = |u|^2|w|^2 - (u.w)^2;
// F < 0 iff v is strictly inside the ball whose great circle is the
// circumcircle of abc
QMN int facedot_exact(const double* a, const double* b, const double* c, const double* v, int* err) {
    Z<2> u[3], w[3], q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) { u[k] = zd(b[k], a[k], err); w[k] = zd(c[k], a[k], err); q[k] = zd(v[k], a[k], err); }
    const Z<4> uu = zdot(u, u), ww = zdot(w, w), uw = zdot(u, w);
    const Z<4> qu = zdot(q, u), qw = zdot(q, w), qq = zdot(q, q);
    Z<7> n2 = zsub(zmul<7>(uu, ww), zmul<7>(uw, uw));
    Z<11> F = zmul<11>(n2, qq);
    F = zsub(F, zmul<11>(zmul<7>(qu, ww), zsub(uu, uw)));
    F = zsub(F, zmul<11>(zmul<7>(qw, uu), zsub(ww, uw)));
    return zsign(F);
}
QMD int facedot(const double* a, const double* b, const double* c, const double* v, int* err) {
    double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
    double w0 = c[0] - a[0], w1 = c[1] - a[1], w2 = c[2] - a[2];
    double q0 = v[0] - a[0], q1 = v[1] - a[1], q2 = v[2] - a[2];
    double uu = (u0 * u0 + u1 * u1) + u2 * u2, ww = (w0 * w0 + w1 * w1) + w2 * w2;
    double uw = (u0 * w0 + u1 * w1) + u2 * w2, qu = (q0 * u0 + q1 * u1) + q2 * u2;
    double qw = (q0 * w0 + q1 * w1) + q2 * w2, qq = (q0 * q0 + q1 * q1) + q2 * q2;
    double puw = (fabs(u0 * w0) + fabs(u1 * w1)) + fabs(u2 * w2);
    double pqu = (fabs(q0 * u0) + fabs(q1 * u1)) + fabs(q2 * u2);
    double pqw = (fabs(q0 * w0) + fabs(q1 * w1)) + fabs(q2 * w2);
    double val = (uu * ww - uw * uw) * qq - qu * ww * (uu - uw) - qw * uu * (ww - uw);
    double per = (uu * ww + puw * puw) * qq + pqu * ww * (uu + puw) + pqw * uu * (ww + puw);
    double bound = 16.0 * kEps * per;
    if (val > bound) return 1;
    if (-val > bound) return -1;
    return facedot_exact(a, b, c, v, err);
}


// --------------------------------------------------------- constructions
QMD double snap(double x) { return rint(x * kLat) * kInvLat; }

QMD void midpoint(const double* a, const double* b, double* p) {
    p[0] = snap((a[0] + b[0]) * 0.5);
    p[1] = snap((a[1] + b[1]) * 0.5);
    p[2] = snap((a[2] + b[2]) * 0.5);
}

QMD void tri_cc(const double* a, const double* b, const double* c, double* p) {
    double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
    double w0 = c[0] - a[0], w1 = c[1] - a[1], w2 = c[2] - a[2];
    double n0 = u1 * w2 - u2 * w1;
    double n1 = u2 * w0 - u0 * w2;
    double n2 = u0 * w1 - u1 * w0;
    double uu = (u0 * u0 + u1 * u1) + u2 * u2;
    double ww = (w0 * w0 + w1 * w1) + w2 * w2;
    double m0 = uu * w0 - ww * u0;
    double m1 = uu * w1 - ww * u1;
    double m2 = uu * w2 - ww * u2;
    double N0 = m1 * n2 - m2 * n1;
    double N1 = m2 * n0 - m0 * n2;
    double N2 = m0 * n1 - m1 * n0;
    double D = 2.0 * ((n0 * n0 + n1 * n1) + n2 * n2);
    p[0] = snap(a[0] + N0 / D);
    p[1] = snap(a[1] + N1 / D);
    p[2] = snap(a[2] + N2 / D);
}

// circumcentre (rounded) and squared circumradius q.q (unrounded)
QMD void tet_cc(const double* a, const double* b, const double* c, const double* d, double* p,
                double& R2) {
    double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
    double v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
    double w0 = d[0] - a[0], w1 = d[1] - a[1], w2 = d[2] - a[2];
    double uu = (u0 * u0 + u1 * u1) + u2 * u2;
    double vv = (v0 * v0 + v1 * v1) + v2 * v2;
    double ww = (w0 * w0 + w1 * w1) + w2 * w2;
    double vw0 = v1 * w2 - v2 * w1, vw1 = v2 * w0 - v0 * w2, vw2 = v0 * w1 - v1 * w0;
    double wu0 = w1 * u2 - w2 * u1, wu1 = w2 * u0 - w0 * u2, wu2 = w0 * u1 - w1 * u0;
    double uv0 = u1 * v2 - u2 * v1, uv1 = u2 * v0 - u0 * v2, uv2 = u0 * v1 - u1 * v0;
    double D = 2.0 * ((u0 * vw0 + u1 * vw1) + u2 * vw2);
    double q0 = ((uu * vw0 + vv * wu0) + ww * uv0) / D;
    double q1 = ((uu * vw1 + vv * wu1) + ww * uv1) / D;
    double q2 = ((uu * vw2 + vv * wu2) + ww * uv2) / D;
    R2 = (q0 * q0 + q1 * q1) + q2 * q2;
    p[0] = snap(a[0] + q0);
    p[1] = snap(a[1] + q1);
    p[2] = snap(a[2] + q2);
}

QMD double d2(const double* a, const double* b) {
    double x = b[0] - a[0], y = b[1] - a[1], z = b[2] - a[2];
    return (x * x + y * y) + z * z;
}

// radius-edge test: R^2 > (B*B) * l^2_min (vertices in ascending id order)
QMD bool is_bad(const double* a, const double* b, const double* c, const double* d, double B2) {
    double p[3], R2;
    tet_cc(a, b, c, d, p, R2);
    double l2 = d2(a, b);
    double e;
    e = d2(a, c); if (e < l2) l2 = e;
    e = d2(a, d); if (e < l2) l2 = e;
    e = d2(b, c); if (e < l2) l2 = e;
    e = d2(b, d); if (e < l2) l2 = e;
    e = d2(c, d); if (e < l2) l2 = e;
    return R2 > B2 * l2;
}

// ------------------------------------------------------------- priorities
// splitmix64 finaliser (Steele, Lea, Flood 2014) chained over sorted ids
QMD uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
QMD uint64_t prio_key(int cls, const int* ids, int n) {
    uint64_t h = 0x9E3779B97F4A7C15ull * (uint64_t)(cls + 1);
    for (int i = 0; i < n; ++i) h = mix64(h ^ (uint64_t)(uint32_t)ids[i]);
    return h;
}

}  // namespace qm
