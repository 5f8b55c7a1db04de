// qm_geom.h -- device geometry for the refinement kernels (gfx950).
//
// Exact predicates: each is an FP64 evaluation with a semi-static error bound
// (error <= c * eps * permanent, Shewchuk 1997, "Adaptive precision
// floating-point arithmetic and fast robust geometric predicates", Sec. 4),
// and, when the sign is not certain, an exact evaluation in floating-point
// expansion arithmetic (same paper, Sec. 2: TWO-SUM, TWO-PRODUCT via FMA,
// FAST-EXPANSION-SUM and SCALE-EXPANSION with zero elimination).
//
// Buffer sizes of the exact paths.  All coordinates are multiples of 2^-53.
// A zero-eliminated nonoverlapping expansion whose value is a multiple of
// 2^L and below 2^H in magnitude has at most H - L + 1 components (the
// components occupy disjoint bit ranges inside [L, H]).  For points of the
// unit cube a degree-d form has L = -53 d and H <= 7, which bounds every
// intermediate of insphere (d = 5) by 273 and of the equatorial-ball test
// (d = 6) by 326 components.  orient3d and orient2d accept any finite point
// (the walks may aim outside the cube) and use the classical length bounds.
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

// error flag raised by an exact path whose precondition fails (never
// expected; reported by the host as an internal error)
__device__ int g_geom_error;

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
                              double* tmp, int cap) {
    int n = 0;
    for (int j = 0; j < bn; ++j) {
        int sn = exp_scale(an, a, b[j], s);
        int m = exp_sum(n, out, sn, s, tmp);
        if (m > cap) { atomicOr(&g_geom_error, 1); m = cap; }
        exp_copy(m, tmp, out);
        n = m;
    }
    return n;
}

// -------------------------------------------------------------- orient3d
// sign of det[b-a; c-a; d-a]
QMN int orient3d_exact(const double* a, const double* b, const double* c, const double* d) {
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
        int n1 = exp_mul(vn[k1], v[k1], wn[k2], w[k2], p1, s, tmp, 8);
        int n2 = exp_mul(vn[k2], v[k2], wn[k1], w[k1], p2, s, tmp, 8);
        exp_neg(n2, p2);
        int mnn = exp_sum(n1, p1, n2, p2, mn);
        int tn = exp_mul(mnn, mn, un[k], u[k], t, s, tmp, 64);
        int m = exp_sum(an, acc, tn, t, tmp);
        exp_copy(m, tmp, acc);
        an = m;
    }
    return exp_sign(an, acc);
}

QMD int orient3d(const double* a, const double* b, const double* c, const double* d) {
    double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
    double v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
    double w0 = d[0] - a[0], w1 = d[1] - a[1], w2 = d[2] - a[2];
    double m0a = v1 * w2, m0b = v2 * w1, m1a = v2 * w0, m1b = v0 * w2, m2a = v0 * w1, m2b = v1 * w0;
    double det = u0 * (m0a - m0b) + u1 * (m1a - m1b) + u2 * (m2a - m2b);
    double per = fabs(u0) * (fabs(m0a) + fabs(m0b)) + fabs(u1) * (fabs(m1a) + fabs(m1b))
               + fabs(u2) * (fabs(m2a) + fabs(m2b));
    double bound = (7.0 + 56.0 * kEps) * kEps * per;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient3d_exact(a, b, c, d);
}

// -------------------------------------------------------------- orient2d
// 2D orientation after dropping coordinate `ax` (kept: ax+1, ax+2 mod 3)
QMN int orient2d_exact(int ax, const double* a, const double* b, const double* c) {
    int i = (ax + 1) % 3, j = (ax + 2) % 3;
    double ux[2], uy[2], vx[2], vy[2];
    int uxn = exp_diff(b[i], a[i], ux), uyn = exp_diff(b[j], a[j], uy);
    int vxn = exp_diff(c[i], a[i], vx), vyn = exp_diff(c[j], a[j], vy);
    double p1[8], p2[8], s[4], tmp[16], out[16];
    int n1 = exp_mul(uxn, ux, vyn, vy, p1, s, tmp, 8);
    int n2 = exp_mul(uyn, uy, vxn, vx, p2, s, tmp, 8);
    exp_neg(n2, p2);
    int n = exp_sum(n1, p1, n2, p2, out);
    return exp_sign(n, out);
}

QMD int orient2d(int ax, const double* a, const double* b, const double* c) {
    int i = (ax + 1) % 3, j = (ax + 2) % 3;
    double ux = b[i] - a[i], uy = b[j] - a[j], vx = c[i] - a[i], vy = c[j] - a[j];
    double l = ux * vy, r = uy * vx;
    double det = l - r;
    double bound = (3.0 + 16.0 * kEps) * kEps * (fabs(l) + fabs(r));
    if (det > bound) return 1;
    if (-det > bound) return -1;
    return orient2d_exact(ax, a, b, c);
}

// exact differences of two points of the unit cube (lattice): one component
QMD double ediff(double x, double y) {
    double h, l;
    two_diff(x, y, h, l);
    if (l != 0.0) atomicOr(&g_geom_error, 2);
    return h;
}

// -------------------------------------------------------------- insphere
// > 0 iff e is strictly inside the circumsphere of positively oriented abcd;
// value = -det[[a-e, |a-e|^2], ..., [d-e, |d-e|^2]]
QMN int insphere_exact(const double* a, const double* b, const double* c, const double* d,
                       const double* e) {
    const double* r[4] = {a, b, c, d};
    double m[4][3];
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 3; ++k) m[i][k] = ediff(r[i][k], e[k]);
    constexpr int CAP = 288;
    double acc[CAP], tmp[CAP], term[CAP], s[64];
    int an = 0;
    for (int i = 0; i < 4; ++i) {
        // lift of row i: x^2 + y^2 + z^2 (<= 6 components)
        double lift[6], sq[2], l2[6];
        int ln = 0;
        for (int k = 0; k < 3; ++k) {
            double x, y;
            two_prod(m[i][k], m[i][k], x, y);
            int qn = 0;
            if (y != 0.0) sq[qn++] = y;
            if (x != 0.0) sq[qn++] = x;
            int nn = exp_sum(ln, lift, qn, sq, l2);
            exp_copy(nn, l2, lift);
            ln = nn;
        }
        // 3x3 minor of the other rows (<= 24 components)
        int rr[3], q = 0;
        for (int s2 = 0; s2 < 4; ++s2) if (s2 != i) rr[q++] = s2;
        double mn[24], mt[24], p[4], t8[8];
        int mnn = 0;
        for (int k = 0; k < 3; ++k) {
            int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
            double x1, y1, x2, y2;
            two_prod(m[rr[1]][k1], m[rr[2]][k2], x1, y1);
            two_prod(m[rr[1]][k2], m[rr[2]][k1], x2, y2);
            double e1[2], e2[2];
            int n1 = 0, n2 = 0;
            if (y1 != 0.0) e1[n1++] = y1;
            if (x1 != 0.0) e1[n1++] = x1;
            if (y2 != 0.0) e2[n2++] = -y2;
            if (x2 != 0.0) e2[n2++] = -x2;
            int pn = exp_sum(n1, e1, n2, e2, p);
            int tn = exp_scale(pn, p, m[rr[0]][k], t8);
            int nn = exp_sum(mnn, mn, tn, t8, mt);
            exp_copy(nn, mt, mn);
            mnn = nn;
        }
        int tn = exp_mul(mnn, mn, ln, lift, term, s, tmp, CAP);
        if ((i + 3) & 1) exp_neg(tn, term);
        int nn = exp_sum(an, acc, tn, term, tmp);
        if (nn > CAP) { atomicOr(&g_geom_error, 4); nn = CAP; }
        exp_copy(nn, tmp, acc);
        an = nn;
    }
    return -exp_sign(an, acc);
}

QMD int insphere(const double* a, const double* b, const double* c, const double* d, const double* e) {
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
    return insphere_exact(a, b, c, d, e);
}

// ------------------------------------------------------ segment encroach
// sign of (v-a).(v-b); negative iff v strictly inside the diametral ball
QMN int segdot_exact(const double* a, const double* b, const double* v) {
    double acc[8], tmp[8];
    int an = 0;
    for (int k = 0; k < 3; ++k) {
        double x, y;
        two_prod(ediff(v[k], a[k]), ediff(v[k], b[k]), x, y);
        double e[2];
        int n = 0;
        if (y != 0.0) e[n++] = y;
        if (x != 0.0) e[n++] = x;
        int nn = exp_sum(an, acc, n, e, tmp);
        exp_copy(nn, tmp, acc);
        an = nn;
    }
    return exp_sign(an, acc);
}
QMD int segdot(const double* a, const double* b, const double* v) {
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
    return segdot_exact(a, b, v);
}

// ----------------------------------------------------- face (equatorial) encroach
// sign of F = |n|^2|q|^2 - (q.u)|w|^2(|u|^2 - u.w) - (q.w)|u|^2(|w|^2 - u.w),
// u = b-a, w = c-a, q = v-a: F < 0 iff v strictly inside the ball whose
// great circle is the circumcircle of abc.
QMD int dot_exp(const double* x, const double* y, double* out) {   // <= 6 components
    double tmp[6];
    int n = 0;
    for (int k = 0; k < 3; ++k) {
        double h, l;
        two_prod(x[k], y[k], h, l);
        double e[2];
        int m = 0;
        if (l != 0.0) e[m++] = l;
        if (h != 0.0) e[m++] = h;
        int nn = exp_sum(n, out, m, e, tmp);
        exp_copy(nn, tmp, out);
        n = nn;
    }
    return n;
}
QMN int facedot_exact(const double* a, const double* b, const double* c, const double* v) {
    double u[3], w[3], q[3];
    for (int k = 0; k < 3; ++k) { u[k] = ediff(b[k], a[k]); w[k] = ediff(c[k], a[k]); q[k] = ediff(v[k], a[k]); }
    double uu[6], ww[6], uw[6], qu[6], qw[6], qq[6], nuwv[6];
    int nuu = dot_exp(u, u, uu), nww = dot_exp(w, w, ww), nuw = dot_exp(u, w, uw);
    int nqu = dot_exp(q, u, qu), nqw = dot_exp(q, w, qw), nqq = dot_exp(q, q, qq);
    exp_copy(nuw, uw, nuwv);
    exp_neg(nuw, nuwv);
    constexpr int CAP = 336;   // span bound of a degree-6 form (see header)
    double s[CAP], tmp[CAP], R[CAP], T[CAP], X1[80], X2[80], S[12];
    // T0 = (uu ww - uw uw) qq
    int n1 = exp_mul(nuu, uu, nww, ww, X1, s, tmp, 80);
    int n2 = exp_mul(nuw, uw, nuw, uw, X2, s, tmp, 80);
    exp_neg(n2, X2);
    int nt = exp_sum(n1, X1, n2, X2, T);
    int nr = exp_mul(nt, T, nqq, qq, R, s, tmp, CAP);
    // - (q.u) ww (uu - uw)
    int ns = exp_sum(nuu, uu, nuw, nuwv, S);
    n1 = exp_mul(nqu, qu, nww, ww, X1, s, tmp, 80);
    nt = exp_mul(n1, X1, ns, S, T, s, tmp, CAP);
    exp_neg(nt, T);
    int m = exp_sum(nr, R, nt, T, tmp);
    if (m > CAP) { atomicOr(&g_geom_error, 8); m = CAP; }
    exp_copy(m, tmp, R);
    nr = m;
    // - (q.w) uu (ww - uw)
    ns = exp_sum(nww, ww, nuw, nuwv, S);
    n1 = exp_mul(nqw, qw, nuu, uu, X1, s, tmp, 80);
    nt = exp_mul(n1, X1, ns, S, T, s, tmp, CAP);
    exp_neg(nt, T);
    m = exp_sum(nr, R, nt, T, tmp);
    if (m > CAP) { atomicOr(&g_geom_error, 8); m = CAP; }
    return exp_sign(m, tmp);
}

QMD int facedot(const double* a, const double* b, const double* c, const double* v) {
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
    return facedot_exact(a, b, c, v);
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
