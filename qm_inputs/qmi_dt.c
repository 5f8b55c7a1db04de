/*
 * qmi_dt.c -- input preparation for the refinement workloads: the Delaunay
 * tetrahedralisation of a lattice point set in the unit cube.
 *
 * The refinement problem (Section 1 of the paper) takes a CDT of the PLC as
 * input.  For the synthetic workloads the initial CDT is the Delaunay
 * tetrahedralisation of the points, so this file builds one.  It is input
 * preparation only: neither the oracle nor the GPU library links it, and it
 * carries its own exact arithmetic (fixed-width integers) so that no code is
 * shared with either of them.
 *
 * Contract:
 *   - points are multiples of 2^-53 in [0,1]^3 (the coordinate lattice);
 *   - points 0..7 are the cube corners, corner i = (i&1, (i>>1)&1, (i>>2)&1);
 *   - points 8.. lie strictly inside the cube and are distinct.
 * Ties (five cospherical points) are broken by symbolic perturbation of the
 * lifted coordinate, the newest (highest id) point receiving the dominant
 * infinitesimal; points are inserted in id order, so the inserted point is
 * always the newest and a tie means "outside".  The corner triangulation is
 * the perturbed Delaunay triangulation of the 8 corners, found by brute force.
 */
/* The builder's working state is thread-local: independent calls may run
   on several host threads at once. */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ---------------- fixed-width signed integers (11 x 32-bit limbs) -------- */
#define GL 11
typedef struct { int neg; uint32_t m[GL]; } gint;

static void g_set(gint* r, int64_t v) {
    memset(r, 0, sizeof *r);
    uint64_t u;
    if (v < 0) { r->neg = 1; u = (uint64_t)(-(v + 1)) + 1u; } else u = (uint64_t)v;
    r->m[0] = (uint32_t)u; r->m[1] = (uint32_t)(u >> 32);
}
static int g_cmpmag(const gint* a, const gint* b) {
    for (int i = GL - 1; i >= 0; --i) {
        if (a->m[i] != b->m[i]) return a->m[i] < b->m[i] ? -1 : 1;
    }
    return 0;
}
static int g_iszero(const gint* a) {
    for (int i = 0; i < GL; ++i) if (a->m[i]) return 0;
    return 1;
}
static int g_sign(const gint* a) { return g_iszero(a) ? 0 : (a->neg ? -1 : 1); }
static void g_addmag(uint32_t* r, const uint32_t* a, const uint32_t* b) {
    uint64_t c = 0;
    for (int i = 0; i < GL; ++i) { c += (uint64_t)a[i] + b[i]; r[i] = (uint32_t)c; c >>= 32; }
}
static void g_submag(uint32_t* r, const uint32_t* a, const uint32_t* b) { /* |a|>=|b| */
    int64_t br = 0;
    for (int i = 0; i < GL; ++i) {
        int64_t d = (int64_t)a[i] - b[i] - br;
        br = d < 0; if (d < 0) d += ((int64_t)1 << 32);
        r[i] = (uint32_t)d;
    }
}
static void g_add(gint* r, const gint* a, const gint* b) {
    gint t;
    memset(&t, 0, sizeof t);
    if (a->neg == b->neg) { g_addmag(t.m, a->m, b->m); t.neg = a->neg; }
    else if (g_cmpmag(a, b) >= 0) { g_submag(t.m, a->m, b->m); t.neg = a->neg; }
    else { g_submag(t.m, b->m, a->m); t.neg = b->neg; }
    if (g_iszero(&t)) t.neg = 0;
    *r = t;
}
static void g_sub(gint* r, const gint* a, const gint* b) { gint nb = *b; nb.neg = !nb.neg; g_add(r, a, &nb); }
static void g_mul(gint* r, const gint* a, const gint* b) {
    uint64_t acc[2 * GL];
    memset(acc, 0, sizeof acc);
    for (int i = 0; i < GL; ++i) {
        if (!a->m[i]) continue;
        uint64_t carry = 0;
        for (int j = 0; j + i < GL; ++j) {
            uint64_t cur = acc[i + j] + (uint64_t)a->m[i] * b->m[j] + carry;
            acc[i + j] = cur & 0xffffffffu; carry = cur >> 32;
        }
    }
    gint t; memset(&t, 0, sizeof t);
    for (int i = 0; i < GL; ++i) t.m[i] = (uint32_t)acc[i];
    t.neg = g_iszero(&t) ? 0 : (a->neg ^ b->neg);
    *r = t;
}

/* lattice coordinate -> integer (x * 2^53 is an integer <= 2^53) */
static int64_t lat(double x) { return (int64_t)ldexp(x, 53); }

/* ---------------- predicates ------------------------------------------- */
static _Thread_local const double* P;   /* coordinates, 3 per point */

/* orient3d(a,b,c,d) = sign det[b-a; c-a; d-a] */
static int orient_exact(int a, int b, int c, int d) {
    gint m[3][3];
    const int o[3] = {b, c, d};
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) g_set(&m[r][k], lat(P[3 * o[r] + k]) - lat(P[3 * a + k]));
    gint t1, t2, s, acc;
    g_set(&acc, 0);
    for (int k = 0; k < 3; ++k) {
        int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        g_mul(&t1, &m[1][k1], &m[2][k2]);
        g_mul(&t2, &m[1][k2], &m[2][k1]);
        g_sub(&s, &t1, &t2);
        g_mul(&t1, &m[0][k], &s);
        g_add(&acc, &acc, &t1);
    }
    return g_sign(&acc);
}
static int orient3d(int a, int b, int c, int d) {
    const double* A = P + 3 * a; const double* B = P + 3 * b;
    const double* C = P + 3 * c; const double* D = P + 3 * d;
    double u[3], v[3], w[3];
    for (int k = 0; k < 3; ++k) { u[k] = B[k] - A[k]; v[k] = C[k] - A[k]; w[k] = D[k] - A[k]; }
    double det = u[0] * (v[1] * w[2] - v[2] * w[1]) + u[1] * (v[2] * w[0] - v[0] * w[2])
               + u[2] * (v[0] * w[1] - v[1] * w[0]);
    double per = fabs(u[0]) * (fabs(v[1] * w[2]) + fabs(v[2] * w[1]))
               + fabs(u[1]) * (fabs(v[2] * w[0]) + fabs(v[0] * w[2]))
               + fabs(u[2]) * (fabs(v[0] * w[1]) + fabs(v[1] * w[0]));
    /* differences of lattice points in [0,1] are exact; 1e-12 is a very
       loose bound on the rounding of the remaining five operations */
    if (det > 1e-12 * per) return 1;
    if (det < -1e-12 * per) return -1;
    return orient_exact(a, b, c, d);
}

/* insphere: > 0 iff e strictly inside the sphere of positively oriented abcd */
static int insphere_exact(int a, int b, int c, int d, int e) {
    const int o[4] = {a, b, c, d};
    gint m[4][4];
    for (int r = 0; r < 4; ++r) {
        gint sq, t;
        g_set(&m[r][3], 0);
        for (int k = 0; k < 3; ++k) {
            g_set(&m[r][k], lat(P[3 * o[r] + k]) - lat(P[3 * e + k]));
            g_mul(&sq, &m[r][k], &m[r][k]);
            g_add(&t, &m[r][3], &sq); m[r][3] = t;
        }
    }
    /* 4x4 determinant by expansion along the lift column */
    gint acc; g_set(&acc, 0);
    for (int r = 0; r < 4; ++r) {
        int rr[3], q = 0;
        for (int s = 0; s < 4; ++s) if (s != r) rr[q++] = s;
        gint minor, t1, t2, s3, acc3; g_set(&acc3, 0);
        for (int k = 0; k < 3; ++k) {
            int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
            g_mul(&t1, &m[rr[1]][k1], &m[rr[2]][k2]);
            g_mul(&t2, &m[rr[1]][k2], &m[rr[2]][k1]);
            g_sub(&s3, &t1, &t2);
            g_mul(&t1, &m[rr[0]][k], &s3);
            g_add(&acc3, &acc3, &t1);
        }
        minor = acc3;
        g_mul(&t1, &m[r][3], &minor);
        /* cofactor sign for (row r, column 3): (-1)^(r+3) */
        if ((r + 3) & 1) g_sub(&acc, &acc, &t1); else g_add(&acc, &acc, &t1);
    }
    /* acc = det[a-e, |a-e|^2; ...] which is positive when e is inside the
       sphere of a negatively oriented tet; flip for positive orientation */
    return -g_sign(&acc);
}
static int insphere_raw(int a, int b, int c, int d, int e) {
    const int o[4] = {a, b, c, d};
    double m[4][4], pm[4][4];
    for (int r = 0; r < 4; ++r) {
        double l = 0;
        for (int k = 0; k < 3; ++k) { m[r][k] = P[3 * o[r] + k] - P[3 * e + k]; l += m[r][k] * m[r][k]; }
        m[r][3] = l;
        for (int k = 0; k < 4; ++k) pm[r][k] = fabs(m[r][k]);
    }
    double det = 0, per = 0;
    for (int r = 0; r < 4; ++r) {
        int rr[3], q = 0;
        for (int s = 0; s < 4; ++s) if (s != r) rr[q++] = s;
        double d3 = 0, p3 = 0;
        for (int k = 0; k < 3; ++k) {
            int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
            d3 += m[rr[0]][k] * (m[rr[1]][k1] * m[rr[2]][k2] - m[rr[1]][k2] * m[rr[2]][k1]);
            p3 += pm[rr[0]][k] * (pm[rr[1]][k1] * pm[rr[2]][k2] + pm[rr[1]][k2] * pm[rr[2]][k1]);
        }
        double t = m[r][3] * d3;
        if ((r + 3) & 1) det -= t; else det += t;
        per += pm[r][3] * p3;
    }
    if (det > 1e-11 * per) return -1;   /* det>0: inside a negatively oriented tet */
    if (det < -1e-11 * per) return 1;
    return insphere_exact(a, b, c, d, e);
}

/* symbolic perturbation of the lift: sign of the perturbed insphere value */
static int insphere_sos(int a, int b, int c, int d, int e) {
    int s = insphere_raw(a, b, c, d, e);
    if (s) return s;
    int ids[5] = {a, b, c, d, e};
    /* visit points by descending id */
    for (int it = 0; it < 5; ++it) {
        int best = -1;
        for (int k = 0; k < 5; ++k)
            if (ids[k] >= 0 && (best < 0 || ids[k] > ids[best])) best = k;
        int x = ids[best];
        ids[best] = -1;
        int coef;
        if (x == e) coef = -orient3d(a, b, c, d);
        else if (x == a) coef = orient3d(e, b, c, d);
        else if (x == b) coef = orient3d(a, e, c, d);
        else if (x == c) coef = orient3d(a, b, e, d);
        else coef = orient3d(a, b, c, e);
        if (coef) return coef;
    }
    return 0;
}

/* ---------------- triangulation ---------------------------------------- */
typedef struct { int v[4]; int adj[4]; } Tet;
static _Thread_local Tet* T; static _Thread_local int nT, capT;
static _Thread_local int* freel; static _Thread_local int nfree, capfree;
static _Thread_local int* dead;   /* 1 if slot is free */

/* inward face triples: orient3d(face, opposite vertex) > 0 */
static const int FI[4][3] = {{1, 3, 2}, {0, 2, 3}, {0, 3, 1}, {0, 1, 2}};

static _Thread_local unsigned char* mark;            /* per tet: 1 in cavity, 2 tested outside */

static int new_tet(void) {
    if (nfree) { int t = freel[--nfree]; dead[t] = 0; return t; }
    if (nT == capT) {
        int old = capT;
        capT = capT ? 2 * capT : 1024;
        T = (Tet*)realloc(T, sizeof(Tet) * (size_t)capT);
        dead = (int*)realloc(dead, sizeof(int) * (size_t)capT);
        mark = (unsigned char*)realloc(mark, (size_t)capT);
        memset(mark + old, 0, (size_t)(capT - old));
    }
    dead[nT] = 0;
    return nT++;
}
static void free_tet(int t) {
    if (nfree == capfree) { capfree = capfree ? 2 * capfree : 1024; freel = (int*)realloc(freel, sizeof(int) * (size_t)capfree); }
    freel[nfree++] = t; dead[t] = 1;
}

static uint64_t ekey(int a, int b) {
    if (a > b) { int t = a; a = b; b = t; }
    return ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
}

/* link tets by matching shared faces among a list (brute force) */
static int link_faces(int* list, int n) {
    for (int i = 0; i < n; ++i) {
        Tet* ti = &T[list[i]];
        for (int f = 0; f < 4; ++f) {
            if (ti->adj[f] != -2) continue;
            int a = ti->v[FI[f][0]], b = ti->v[FI[f][1]], c = ti->v[FI[f][2]];
            int found = 0;
            for (int j = 0; j < n && !found; ++j) {
                if (j == i) continue;
                Tet* tj = &T[list[j]];
                for (int g = 0; g < 4; ++g) {
                    int x = tj->v[FI[g][0]], y = tj->v[FI[g][1]], z = tj->v[FI[g][2]];
                    /* opposite orientation: (a,b,c) vs reversed cyclic of (x,y,z) */
                    if ((a == x && b == z && c == y) || (a == y && b == x && c == z) || (a == z && b == y && c == x)) {
                        ti->adj[f] = (list[j] << 2) | g;
                        tj->adj[g] = (list[i] << 2) | f;
                        found = 1; break;
                    }
                }
            }
            if (!found) ti->adj[f] = -1;
        }
    }
    return 0;
}

static int corner_dt(void) {
    int list[64], n = 0;
    for (int a = 0; a < 8; ++a)
        for (int b = a + 1; b < 8; ++b)
            for (int c = b + 1; c < 8; ++c)
                for (int d = c + 1; d < 8; ++d) {
                    int o = orient3d(a, b, c, d);
                    if (!o) continue;
                    int v[4] = {a, b, c, d};
                    if (o < 0) { v[2] = d; v[3] = c; }
                    int ok = 1;
                    for (int e = 0; e < 8 && ok; ++e) {
                        if (e == a || e == b || e == c || e == d) continue;
                        if (insphere_sos(v[0], v[1], v[2], v[3], e) > 0) ok = 0;
                    }
                    if (ok) {
                        if (n >= 64) return -1;
                        int t = new_tet();
                        for (int k = 0; k < 4; ++k) { T[t].v[k] = v[k]; T[t].adj[k] = -2; }
                        list[n++] = t;
                    }
                }
    link_faces(list, n);
    return n;
}

/* cavity work buffers */
static _Thread_local int *cav, ncav, capcav;
static _Thread_local int *bnd, nbnd, capbnd;          /* boundary faces (t<<2|f) */
static _Thread_local int* touched; static _Thread_local int ntouched, captouched;

static void push(int** arr, int* n, int* cap, int v) {
    if (*n == *cap) { *cap = *cap ? 2 * *cap : 256; *arr = (int*)realloc(*arr, sizeof(int) * (size_t)*cap); }
    (*arr)[(*n)++] = v;
}

/* edge hash for internal linking of new tets */
typedef struct { uint64_t k; int tf; } EH;
static _Thread_local EH* eh; static _Thread_local int ehcap;

static int insert_point(int p, int* start) {
    /* visibility walk */
    int t = *start, steps = 0;
    for (;;) {
        if (++steps > 100000000) return -3;
        int moved = 0;
        for (int f = 0; f < 4; ++f) {
            const int* v = T[t].v;
            if (orient3d(v[FI[f][0]], v[FI[f][1]], v[FI[f][2]], p) < 0) {
                int n = T[t].adj[f];
                if (n < 0) return -4; /* point outside the hull */
                t = n >> 2; moved = 1; break;
            }
        }
        if (!moved) break;
    }
    /* cavity BFS */
    ncav = 0; nbnd = 0; ntouched = 0;
    if (insphere_sos(T[t].v[0], T[t].v[1], T[t].v[2], T[t].v[3], p) <= 0) return -5;
    push(&cav, &ncav, &capcav, t); mark[t] = 1; push(&touched, &ntouched, &captouched, t);
    for (int i = 0; i < ncav; ++i) {
        int c = cav[i];
        for (int f = 0; f < 4; ++f) {
            int n = T[c].adj[f];
            if (n < 0) { push(&bnd, &nbnd, &capbnd, (c << 2) | f); continue; }
            int nt = n >> 2;
            if (mark[nt] == 0) {
                const int* v = T[nt].v;
                mark[nt] = insphere_sos(v[0], v[1], v[2], v[3], p) > 0 ? 1 : 2;
                push(&touched, &ntouched, &captouched, nt);
                if (mark[nt] == 1) push(&cav, &ncav, &capcav, nt);
            }
            if (mark[nt] == 2) push(&bnd, &nbnd, &capbnd, (c << 2) | f);
        }
    }
    /* new tets from boundary faces */
    int nb = nbnd;
    int* newt = (int*)malloc(sizeof(int) * (size_t)nb);
    int* oldadj = (int*)malloc(sizeof(int) * (size_t)nb);
    int fv[3];
    int (*faces)[3] = (int(*)[3])malloc(sizeof(int) * 3 * (size_t)nb);
    for (int i = 0; i < nb; ++i) {
        int c = bnd[i] >> 2, f = bnd[i] & 3;
        for (int k = 0; k < 3; ++k) fv[k] = T[c].v[FI[f][k]];
        memcpy(faces[i], fv, sizeof fv);
        oldadj[i] = T[c].adj[f];
        if (orient3d(fv[0], fv[1], fv[2], p) <= 0) { free(newt); free(oldadj); free(faces); return -6; }
    }
    for (int i = 0; i < ntouched; ++i) mark[touched[i]] = 0;
    for (int i = 0; i < ncav; ++i) free_tet(cav[i]);
    for (int i = 0; i < nb; ++i) {
        int s = new_tet();
        newt[i] = s;
        T[s].v[0] = faces[i][0]; T[s].v[1] = faces[i][1]; T[s].v[2] = faces[i][2]; T[s].v[3] = p;
        T[s].adj[3] = oldadj[i];
        if (oldadj[i] >= 0) T[oldadj[i] >> 2].adj[oldadj[i] & 3] = (s << 2) | 3;
    }
    /* internal links: face of new tet opposite face vertex k contains p and the other two */
    int need = 1;
    while (need < 6 * nb) need <<= 1;
    if (need > ehcap) { ehcap = need; eh = (EH*)realloc(eh, sizeof(EH) * (size_t)ehcap); }
    for (int i = 0; i < need; ++i) eh[i].k = 0;
    for (int i = 0; i < nb; ++i) {
        for (int k = 0; k < 3; ++k) {
            int x = faces[i][(k + 1) % 3], y = faces[i][(k + 2) % 3];
            uint64_t key = ekey(x, y) + 1;
            uint64_t h = (key * 0x9E3779B97F4A7C15ull) & (uint64_t)(need - 1);
            for (;;) {
                if (eh[h].k == 0) { eh[h].k = key; eh[h].tf = (newt[i] << 2) | k; break; }
                if (eh[h].k == key) {
                    int o = eh[h].tf;
                    T[newt[i]].adj[k] = o;
                    T[o >> 2].adj[o & 3] = (newt[i] << 2) | k;
                    eh[h].k = ~0ull; /* consumed */
                    break;
                }
                h = (h + 1) & (uint64_t)(need - 1);
            }
        }
    }
    *start = newt[0];
    free(newt); free(oldadj); free(faces);
    return 0;
}

/*
 * qmi_delaunay: build the Delaunay tetrahedralisation.
 *   n, xyz   : points (see contract above)
 *   out_nt   : number of tets written
 *   out_tets : caller buffer of cap*4 ints (positively oriented)
 *   out_adj  : caller buffer of cap*4 ints (t<<2|f, -1 on the hull)
 * Returns 0, or a negative code: -1 bad corners, -2 capacity, -3 walk,
 * -4 point outside, -5/-6 degenerate input (duplicate or coplanar case).
 */
int qmi_delaunay(int n, const double* xyz, int cap, int* out_nt, int* out_tets, int* out_adj) {
    P = xyz;
    T = NULL; nT = capT = 0; freel = NULL; nfree = capfree = 0; dead = NULL; mark = NULL;
    int rc = 0;
    if (n < 8) return -1;
    int nc = corner_dt();
    if (nc <= 0) return -1;
    int start = 0;
    for (int p = 8; p < n; ++p) {
        rc = insert_point(p, &start);
        if (rc) goto done;
    }
    /* compact */
    {
        int* remap = (int*)malloc(sizeof(int) * (size_t)(nT ? nT : 1));
        int m = 0;
        for (int t = 0; t < nT; ++t) remap[t] = dead[t] ? -1 : m++;
        if (m > cap) { free(remap); rc = -2; goto done; }
        for (int t = 0; t < nT; ++t) {
            if (dead[t]) continue;
            int s = remap[t];
            for (int k = 0; k < 4; ++k) {
                out_tets[4 * s + k] = T[t].v[k];
                int a = T[t].adj[k];
                out_adj[4 * s + k] = a < 0 ? -1 : ((remap[a >> 2] << 2) | (a & 3));
            }
        }
        *out_nt = m;
        free(remap);
    }
done:
    free(T); free(freel); free(dead); free(mark);
    free(cav); cav = NULL; ncav = capcav = 0;
    free(bnd); bnd = NULL; nbnd = capbnd = 0;
    free(touched); touched = NULL; ntouched = captouched = 0;
    free(eh); eh = NULL; ehcap = 0;
    T = NULL; freel = NULL; dead = NULL; mark = NULL;
    return rc;
}
