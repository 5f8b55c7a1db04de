/*
 * qmo_exact.h -- exact geometric predicates and canonical FP64 constructions
 * of the ORACLE (test infrastructure; see qmo.c).  Nothing outside oracle/
 * includes this file.
 *
 * Exactness: every coordinate is a multiple of 2^-53 (the coordinate lattice
 * of the workloads; splitting points are rounded onto it), so x * 2^53 is an
 * integer and each predicate is the sign of an integer polynomial.  The
 * oracle first evaluates the polynomial in FP64 together with its permanent
 * (the same polynomial over absolute values); when |value| exceeds 1e-10
 * times the permanent -- about a million times the worst-case rounding of
 * these short formulas -- the FP64 sign is certain.  Otherwise the sign is
 * computed with plain schoolbook big-integer arithmetic.
 */
#ifndef QMO_EXACT_H
#define QMO_EXACT_H

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- bignum */
#define BN_MAX 136   /* 32-bit limbs: enough for degree-3 forms of any finite double */

typedef struct { int n; int neg; uint32_t d[BN_MAX]; } bn;

static void bn_fail(void) { abort(); }

static void bn_norm(bn* a) {
    while (a->n > 0 && a->d[a->n - 1] == 0) a->n--;
    if (a->n == 0) a->neg = 0;
}

/* exact integer value of x * 2^53 for a lattice double x */
static void bn_from_lattice(bn* r, double x) {
    memset(r, 0, sizeof *r);
    if (x == 0.0) return;
    int e;
    double m = frexp(fabs(x), &e);             /* |x| = m 2^e, 0.5 <= m < 1 */
    uint64_t M = (uint64_t)ldexp(m, 53);       /* exact 53-bit integer */
    int sh = e;                                /* x 2^53 = M 2^(e) */
    if (sh < 0) {
        if (sh < -63 || (M & ((1ull << -sh) - 1))) bn_fail();   /* off the lattice */
        M >>= -sh; sh = 0;
    }
    int w = sh / 32, b = sh % 32;
    if (w + 3 > BN_MAX) bn_fail();
    unsigned __int128 v = (unsigned __int128)M << b;
    r->d[w] = (uint32_t)v; r->d[w + 1] = (uint32_t)(v >> 32); r->d[w + 2] = (uint32_t)(v >> 64);
    r->n = w + 3; r->neg = x < 0;
    bn_norm(r);
}

static int bn_cmpmag(const bn* a, const bn* b) {
    if (a->n != b->n) return a->n < b->n ? -1 : 1;
    for (int i = a->n - 1; i >= 0; --i)
        if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
    return 0;
}

static void bn_add(bn* r, const bn* a, const bn* b) {
    bn t; memset(&t, 0, sizeof t);
    if (a->neg == b->neg) {
        int n = a->n > b->n ? a->n : b->n;
        uint64_t c = 0;
        for (int i = 0; i < n; ++i) {
            c += (uint64_t)(i < a->n ? a->d[i] : 0) + (i < b->n ? b->d[i] : 0);
            t.d[i] = (uint32_t)c; c >>= 32;
        }
        if (c) { if (n >= BN_MAX) bn_fail(); t.d[n++] = (uint32_t)c; }
        t.n = n; t.neg = a->neg;
    } else {
        const bn *x = a, *y = b;
        if (bn_cmpmag(a, b) < 0) { x = b; y = a; }
        int64_t br = 0;
        for (int i = 0; i < x->n; ++i) {
            int64_t d = (int64_t)x->d[i] - (i < y->n ? y->d[i] : 0) - br;
            br = d < 0; if (br) d += (int64_t)1 << 32;
            t.d[i] = (uint32_t)d;
        }
        t.n = x->n; t.neg = x->neg;
    }
    bn_norm(&t);
    *r = t;
}

static void bn_sub(bn* r, const bn* a, const bn* b) { bn nb = *b; if (nb.n) nb.neg = !nb.neg; bn_add(r, a, &nb); }

static void bn_mul(bn* r, const bn* a, const bn* b) {
    bn t; memset(&t, 0, sizeof t);
    if (a->n == 0 || b->n == 0) { *r = t; return; }
    if (a->n + b->n > BN_MAX) bn_fail();
    for (int i = 0; i < a->n; ++i) {
        uint64_t c = 0;
        for (int j = 0; j < b->n; ++j) {
            uint64_t cur = (uint64_t)t.d[i + j] + (uint64_t)a->d[i] * b->d[j] + c;
            t.d[i + j] = (uint32_t)cur; c = cur >> 32;
        }
        t.d[i + b->n] = (uint32_t)c;
    }
    t.n = a->n + b->n; t.neg = a->neg ^ b->neg;
    bn_norm(&t);
    *r = t;
}

static int bn_sign(const bn* a) { return a->n == 0 ? 0 : (a->neg ? -1 : 1); }

/* ------------------------------------------------------- filter constant */
#define QMO_FILTER 1e-10

static int fsign(double v, double per, int* certain) {
    *certain = 0;
    if (!isfinite(v) || !isfinite(per)) return 0;
    if (v > QMO_FILTER * per) { *certain = 1; return 1; }
    if (v < -QMO_FILTER * per) { *certain = 1; return -1; }
    return 0;
}

/* ------------------------------------------------------------- orient3d */
/* sign of det[b-a; c-a; d-a]: > 0 when (b-a, c-a, d-a) is right-handed */
static int qmo_orient3d(const double* a, const double* b, const double* c, const double* d) {
    double u[3], v[3], w[3];
    for (int k = 0; k < 3; ++k) { u[k] = b[k] - a[k]; v[k] = c[k] - a[k]; w[k] = d[k] - a[k]; }
    double val = u[0] * (v[1] * w[2] - v[2] * w[1]) + u[1] * (v[2] * w[0] - v[0] * w[2])
               + u[2] * (v[0] * w[1] - v[1] * w[0]);
    double per = fabs(u[0]) * (fabs(v[1] * w[2]) + fabs(v[2] * w[1]))
               + fabs(u[1]) * (fabs(v[2] * w[0]) + fabs(v[0] * w[2]))
               + fabs(u[2]) * (fabs(v[0] * w[1]) + fabs(v[1] * w[0]));
    int ok, s = fsign(val, per, &ok);
    if (ok) return s;
    bn A[3], U[3], V[3], W[3], t1, t2, t3, acc;
    for (int k = 0; k < 3; ++k) {
        bn_from_lattice(&A[k], a[k]);
        bn_from_lattice(&t1, b[k]); bn_sub(&U[k], &t1, &A[k]);
        bn_from_lattice(&t1, c[k]); bn_sub(&V[k], &t1, &A[k]);
        bn_from_lattice(&t1, d[k]); bn_sub(&W[k], &t1, &A[k]);
    }
    memset(&acc, 0, sizeof acc);
    for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        bn_mul(&t1, &V[k1], &W[k2]);
        bn_mul(&t2, &V[k2], &W[k1]);
        bn_sub(&t3, &t1, &t2);
        bn_mul(&t1, &U[k], &t3);
        bn_add(&acc, &acc, &t1);
    }
    return bn_sign(&acc);
}

/* ------------------------------------------------------------- insphere */
/* > 0 iff e is strictly inside the circumsphere of positively oriented abcd.
   Value = -det[[a-e, |a-e|^2], [b-e, ...], [c-e, ...], [d-e, ...]]. */
static int qmo_insphere(const double* a, const double* b, const double* c, const double* d,
                        const double* e) {
    const double* r[4] = {a, b, c, d};
    double m[4][4], pm[4][4];
    for (int i = 0; i < 4; ++i) {
        for (int k = 0; k < 3; ++k) m[i][k] = r[i][k] - e[k];
        m[i][3] = (m[i][0] * m[i][0] + m[i][1] * m[i][1]) + m[i][2] * m[i][2];
        for (int k = 0; k < 4; ++k) pm[i][k] = fabs(m[i][k]);
    }
    double det = 0, per = 0;
    for (int i = 0; i < 4; ++i) {
        int rr[3], q = 0;
        for (int s = 0; s < 4; ++s) if (s != i) rr[q++] = s;
        double d3 = 0, p3 = 0;
        for (int k = 0; k < 3; ++k) {
            int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
            d3 += m[rr[0]][k] * (m[rr[1]][k1] * m[rr[2]][k2] - m[rr[1]][k2] * m[rr[2]][k1]);
            p3 += pm[rr[0]][k] * (pm[rr[1]][k1] * pm[rr[2]][k2] + pm[rr[1]][k2] * pm[rr[2]][k1]);
        }
        double t = m[i][3] * d3;
        if ((i + 3) & 1) det -= t; else det += t;
        per += pm[i][3] * p3;
    }
    int ok, s = fsign(-det, per, &ok);
    if (ok) return s;
    bn M[4][4], E[3], t1, t2, t3, acc;
    for (int k = 0; k < 3; ++k) bn_from_lattice(&E[k], e[k]);
    for (int i = 0; i < 4; ++i) {
        memset(&M[i][3], 0, sizeof(bn));
        for (int k = 0; k < 3; ++k) {
            bn_from_lattice(&t1, r[i][k]);
            bn_sub(&M[i][k], &t1, &E[k]);
            bn_mul(&t2, &M[i][k], &M[i][k]);
            bn_add(&M[i][3], &M[i][3], &t2);
        }
    }
    memset(&acc, 0, sizeof acc);
    for (int i = 0; i < 4; ++i) {
        int rr[3], q = 0;
        for (int s2 = 0; s2 < 4; ++s2) if (s2 != i) rr[q++] = s2;
        bn d3; memset(&d3, 0, sizeof d3);
        for (int k = 0; k < 3; ++k) {
            int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
            bn_mul(&t1, &M[rr[1]][k1], &M[rr[2]][k2]);
            bn_mul(&t2, &M[rr[1]][k2], &M[rr[2]][k1]);
            bn_sub(&t3, &t1, &t2);
            bn_mul(&t1, &M[rr[0]][k], &t3);
            bn_add(&d3, &d3, &t1);
        }
        bn_mul(&t1, &M[i][3], &d3);
        if ((i + 3) & 1) bn_sub(&acc, &acc, &t1); else bn_add(&acc, &acc, &t1);
    }
    return -bn_sign(&acc);
}

/* ------------------------------------------------------- orient2d (proj) */
/* 2D orientation after dropping coordinate `axis`; the kept coordinates are
   (axis+1)%3 and (axis+2)%3, in that order. */
static int qmo_orient2d(int axis, const double* a, const double* b, const double* c) {
    int i = (axis + 1) % 3, j = (axis + 2) % 3;
    double ux = b[i] - a[i], uy = b[j] - a[j], vx = c[i] - a[i], vy = c[j] - a[j];
    double val = ux * vy - uy * vx;
    double per = fabs(ux * vy) + fabs(uy * vx);
    int ok, s = fsign(val, per, &ok);
    if (ok) return s;
    bn A0, A1, U0, U1, V0, V1, t1, t2, acc;
    bn_from_lattice(&A0, a[i]); bn_from_lattice(&A1, a[j]);
    bn_from_lattice(&t1, b[i]); bn_sub(&U0, &t1, &A0);
    bn_from_lattice(&t1, b[j]); bn_sub(&U1, &t1, &A1);
    bn_from_lattice(&t1, c[i]); bn_sub(&V0, &t1, &A0);
    bn_from_lattice(&t1, c[j]); bn_sub(&V1, &t1, &A1);
    bn_mul(&t1, &U0, &V1); bn_mul(&t2, &U1, &V0); bn_sub(&acc, &t1, &t2);
    return bn_sign(&acc);
}

/* ------------------------------------------------------- segment encroach */
/* sign of (v-a).(v-b): negative iff v lies strictly inside the diametral
   ball of segment ab. */
static int qmo_segdot(const double* a, const double* b, const double* v) {
    double val = 0, per = 0;
    for (int k = 0; k < 3; ++k) {
        double x = v[k] - a[k], y = v[k] - b[k];
        val += x * y; per += fabs(x * y);
    }
    int ok, s = fsign(val, per, &ok);
    if (ok) return s;
    bn acc, A, Bv, X, Y, t; memset(&acc, 0, sizeof acc);
    for (int k = 0; k < 3; ++k) {
        bn_from_lattice(&t, v[k]);
        bn_from_lattice(&A, a[k]); bn_sub(&X, &t, &A);
        bn_from_lattice(&Bv, b[k]); bn_sub(&Y, &t, &Bv);
        bn_mul(&A, &X, &Y); bn_add(&acc, &acc, &A);
    }
    return bn_sign(&acc);
}

/* ---------------------------------------------------------- face encroach */
/* Sign of F = |n|^2 |q|^2 - (q.u)|w|^2(|u|^2 - u.w) - (q.w)|u|^2(|w|^2 - u.w)
   with u = b-a, w = c-a, q = v-a, n = u x w.  F is half of
   D|q|^2 - 2 q.N (D = 2|n|^2, N = (|u|^2 w - |w|^2 u) x n), i.e. the power of
   v with respect to the equatorial ball of triangle abc times D/2.  v is
   strictly inside that ball iff F < 0. */
static int qmo_facedot(const double* a, const double* b, const double* c, const double* v) {
    double u[3], w[3], q[3];
    for (int k = 0; k < 3; ++k) { u[k] = b[k] - a[k]; w[k] = c[k] - a[k]; q[k] = v[k] - a[k]; }
#define DOT(x, y) ((x[0] * y[0] + x[1] * y[1]) + x[2] * y[2])
#define PDOT(x, y) ((fabs(x[0] * y[0]) + fabs(x[1] * y[1])) + fabs(x[2] * y[2]))
    double uu = DOT(u, u), ww = DOT(w, w), uw = DOT(u, w), qu = DOT(q, u), qw = DOT(q, w), qq = DOT(q, q);
    double puw = PDOT(u, w), pqu = PDOT(q, u), pqw = PDOT(q, w);
#undef DOT
#undef PDOT
    double val = (uu * ww - uw * uw) * qq - qu * ww * (uu - uw) - qw * uu * (ww - uw);
    double per = (uu * ww + puw * puw) * qq + pqu * ww * (uu + puw) + pqw * uu * (ww + puw);
    int ok, s = fsign(val, per, &ok);
    if (ok) return s;
    bn U[3], W[3], Q[3], A, t, t2;
    for (int k = 0; k < 3; ++k) {
        bn_from_lattice(&A, a[k]);
        bn_from_lattice(&t, b[k]); bn_sub(&U[k], &t, &A);
        bn_from_lattice(&t, c[k]); bn_sub(&W[k], &t, &A);
        bn_from_lattice(&t, v[k]); bn_sub(&Q[k], &t, &A);
    }
    bn UU, WW, UW, QU, QW, QQ;
    bn* outs[6] = {&UU, &WW, &UW, &QU, &QW, &QQ};
    bn* xs[6] = {U, W, U, Q, Q, Q};
    bn* ys[6] = {U, W, W, U, W, Q};
    for (int i = 0; i < 6; ++i) {
        memset(outs[i], 0, sizeof(bn));
        for (int k = 0; k < 3; ++k) { bn_mul(&t, &xs[i][k], &ys[i][k]); bn_add(outs[i], outs[i], &t); }
    }
    bn N2, F, T1, T2;
    bn_mul(&t, &UU, &WW); bn_mul(&t2, &UW, &UW); bn_sub(&N2, &t, &t2);
    bn_mul(&F, &N2, &QQ);
    bn_sub(&t, &UU, &UW); bn_mul(&t2, &QU, &WW); bn_mul(&T1, &t2, &t);
    bn_sub(&t, &WW, &UW); bn_mul(&t2, &QW, &UU); bn_mul(&T2, &t2, &t);
    bn_sub(&F, &F, &T1); bn_sub(&F, &F, &T2);
    return bn_sign(&F);
}

/* ------------------------------------------------ canonical constructions */
/* All constructions take the vertices in ascending id order (a = lowest),
   use FP64 with this exact operation order (no contraction), and round the
   result onto the 2^-53 lattice. */
static double qmo_snap(double x) { return ldexp(rint(ldexp(x, 53)), -53); }

static void qmo_midpoint(const double* a, const double* b, double* p) {
    for (int k = 0; k < 3; ++k) p[k] = qmo_snap((a[k] + b[k]) * 0.5);
}

static void qmo_tri_cc(const double* a, const double* b, const double* c, double* p) {
    double u[3], w[3];
    for (int k = 0; k < 3; ++k) { u[k] = b[k] - a[k]; w[k] = c[k] - a[k]; }
    double n0 = u[1] * w[2] - u[2] * w[1];
    double n1 = u[2] * w[0] - u[0] * w[2];
    double n2 = u[0] * w[1] - u[1] * w[0];
    double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    double ww = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
    double m0 = uu * w[0] - ww * u[0];
    double m1 = uu * w[1] - ww * u[1];
    double m2 = uu * w[2] - ww * u[2];
    double N0 = m1 * n2 - m2 * n1;
    double N1 = m2 * n0 - m0 * n2;
    double N2 = m0 * n1 - m1 * n0;
    double D = 2.0 * ((n0 * n0 + n1 * n1) + n2 * n2);
    p[0] = qmo_snap(a[0] + N0 / D);
    p[1] = qmo_snap(a[1] + N1 / D);
    p[2] = qmo_snap(a[2] + N2 / D);
}

/* circumcentre (rounded) and squared circumradius (unrounded q.q) */
static void qmo_tet_cc(const double* a, const double* b, const double* c, const double* d,
                       double* p, double* R2) {
    double u[3], v[3], w[3];
    for (int k = 0; k < 3; ++k) { u[k] = b[k] - a[k]; v[k] = c[k] - a[k]; w[k] = d[k] - a[k]; }
    double uu = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    double vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    double ww = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2];
    double vw[3] = {v[1] * w[2] - v[2] * w[1], v[2] * w[0] - v[0] * w[2], v[0] * w[1] - v[1] * w[0]};
    double wu[3] = {w[1] * u[2] - w[2] * u[1], w[2] * u[0] - w[0] * u[2], w[0] * u[1] - w[1] * u[0]};
    double uv[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    double D = 2.0 * ((u[0] * vw[0] + u[1] * vw[1]) + u[2] * vw[2]);
    double q[3];
    for (int k = 0; k < 3; ++k) q[k] = ((uu * vw[k] + vv * wu[k]) + ww * uv[k]) / D;
    *R2 = (q[0] * q[0] + q[1] * q[1]) + q[2] * q[2];
    for (int k = 0; k < 3; ++k) p[k] = qmo_snap(a[k] + q[k]);
}

static double qmo_d2(const double* a, const double* b) {
    double x = b[0] - a[0], y = b[1] - a[1], z = b[2] - a[2];
    return (x * x + y * y) + z * z;
}

/* radius-edge test of Section 1: circumradius / shortest edge > B, evaluated
   as R^2 > (B*B) * l^2_min in FP64 */
static int qmo_is_bad(const double* a, const double* b, const double* c, const double* d, double B2) {
    double p[3], R2;
    qmo_tet_cc(a, b, c, d, p, &R2);
    const double* v[4] = {a, b, c, d};
    double l2 = qmo_d2(a, b);
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j) {
            double e = qmo_d2(v[i], v[j]);
            if (e < l2) l2 = e;
        }
    return R2 > B2 * l2;
}

/* ------------------------------------------------------ priority keys */
/* splitmix64 finaliser (Steele, Lea and Flood, "Fast splittable
   pseudorandom number generators", 2014) chained over the sorted ids */
static uint64_t qmo_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t qmo_key(int cls, const int* ids, int n) {
    uint64_t h = 0x9E3779B97F4A7C15ull * (uint64_t)(cls + 1);
    for (int i = 0; i < n; ++i) h = qmo_mix64(h ^ (uint64_t)(uint32_t)ids[i]);
    return h;
}

#endif
