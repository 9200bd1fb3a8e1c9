/*
 * CPU oracle for the differentiable light-stage face renderer.
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread.
 * No contraction: every float/double operation below is rounded on its own,
 * in the order written.
 *
 * The estimator follows the paper (Dib et al. 2019):
 *   Face Modeling paragraph - light stage of N oriented area lights with RGB
 *     intensities l_j; morphable geometry (alpha, beta), pose [R t], albedo
 *     (delta), vertex normals n_i, Cook-Torrance reflectance
 *     f_r = k_d f_lambert + k_s f_cook-torrance with a gray specular texture;
 *   Optimization paragraph - p = F(f_r, l_j, alpha, beta, R, t), the
 *     Monte-Carlo estimator of the lighting equation with ray-traced
 *     self-shadows; E_data = sum ||p^T - p^R||^2 (Eq. 1);
 *   Face Modeling paragraph - gradients by differentiable ray tracing with
 *     edge sampling of visibility discontinuities.
 * Readings of points the paper leaves open are fixed in the design notes
 * (Beckmann roughness 0.35, F = 1, k_d = k_s = 1, two-sided surfaces, direct
 * lighting only, box pixel filter, black background).
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846
#define BECKMANN_M 0.35
#define MAXL 64                 /* lights supported by the oracle            */
#define HIT_MARGIN 1e-5f        /* accepted hit point within tri box +- this */
#define BOX_PAD 2e-5f           /* BVH boxes padded by this (culling only)   */
#define SHADOW_TMIN 1e-4f
#define SHADOW_TMAX (1.0f - 1e-4f)
#define EDGE_OFF_PX 1e-3f       /* screen offset of the two silhouette sides */
#define EDGE_OFF_M 2e-5f        /* light-plane offset of the two shadow sides */
#define QSCALE 1048576.0f       /* 2^20: edge weight quantisation            */
#define ORC_REC_WORDS 9         /* int32 words of one decision record        */

/* ------------------------------------------------------------ Philox ---- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
 * 32x32->64 multiplies with key schedule bumped by the Weyl constants. */
void orc_philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                uint32_t c2, uint32_t c3, uint32_t out[4]) {
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static inline float u01(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

/* Camera sample s draws 44 words from counters (s, b, 0, 0), b = 0..10:
 * words 0,1 pixel jitter; words 2+2j, 3+2j light j's (u, v). */
static void camera_words(uint64_t seed, uint32_t s, uint32_t *w /*44*/) {
    for (uint32_t b = 0; b < 11; ++b)
        orc_philox((uint32_t)seed, (uint32_t)(seed >> 32), s, b, 0, 0, w + 4 * b);
}

/* --------------------------------------------------- small vector ops ---- */
typedef struct { float x, y, z; } f3;
typedef struct { double x, y, z; } d3;

static inline f3 fsub(f3 a, f3 b) { f3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static inline float fdot(f3 a, f3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static inline f3 fcross(f3 a, f3 b) {
    f3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
static inline d3 dmk(double x, double y, double z) { d3 r = {x, y, z}; return r; }
static inline d3 dadd(d3 a, d3 b) { return dmk(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline d3 dsub(d3 a, d3 b) { return dmk(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline d3 dscl(d3 a, double s) { return dmk(a.x * s, a.y * s, a.z * s); }
static inline double ddot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline d3 dcross(d3 a, d3 b) {
    return dmk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline double dlen(d3 a) { return sqrt(ddot(a, a)); }
static inline d3 d_of(f3 a) { return dmk(a.x, a.y, a.z); }
/* adjoint of n = v/|v| : returns dL/dv given dL/dn, n and |v| */
static inline d3 dnorm_adj(d3 gn, d3 n, double len) {
    return dscl(dsub(gn, dscl(n, ddot(n, gn))), 1.0 / len);
}
static inline void dacc(double *a, int V, int i, d3 g) {
    a[i] += g.x; a[V + i] += g.y; a[2 * V + i] += g.z;
}

static inline f3 fpos(const orc_scene *s, int i) {
    f3 r = {s->pos[i], s->pos[s->V + i], s->pos[2 * s->V + i]}; return r;
}
static inline d3 dpos(const orc_scene *s, int i) {
    return dmk(s->pos_d[i], s->pos_d[s->V + i], s->pos_d[2 * s->V + i]);
}

/* ---------------------------------------------- morphable model (fp64) -- */
void orc_rotation(const float pose[6], double R[9]) {
    double cx = cos((double)pose[0]), sx = sin((double)pose[0]);
    double cy = cos((double)pose[1]), sy = sin((double)pose[1]);
    double cz = cos((double)pose[2]), sz = sin((double)pose[2]);
    double Rx[9] = {1, 0, 0, 0, cx, -sx, 0, sx, cx};
    double Ry[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy};
    double Rz[9] = {cz, -sz, 0, sz, cz, 0, 0, 0, 1};
    double T[9];
    for (int i = 0; i < 3; ++i)          /* T = Ry Rx */
        for (int j = 0; j < 3; ++j)
            T[3 * i + j] = (Ry[3 * i + 0] * Rx[0 + j] + Ry[3 * i + 1] * Rx[3 + j]) + Ry[3 * i + 2] * Rx[6 + j];
    for (int i = 0; i < 3; ++i)          /* R = Rz T */
        for (int j = 0; j < 3; ++j)
            R[3 * i + j] = (Rz[3 * i + 0] * T[0 + j] + Rz[3 * i + 1] * T[3 + j]) + Rz[3 * i + 2] * T[6 + j];
}

void orc_blend_geometry(int32_t V, int32_t n_id, int32_t n_exp,
                        const float *mean, const float *b_id, const float *b_exp,
                        const float *alpha, const float *beta, const float pose[6],
                        double *v_model, double *v) {
    double R[9];
    orc_rotation(pose, R);
    for (int32_t i = 0; i < V; ++i) {
        double m[3];
        for (int c = 0; c < 3; ++c) {
            size_t e = (size_t)c * V + i;
            double acc = mean[e];
            for (int k = 0; k < n_id; ++k) acc = acc + (double)b_id[(size_t)k * 3 * V + e] * (double)alpha[k];
            for (int k = 0; k < n_exp; ++k) acc = acc + (double)b_exp[(size_t)k * 3 * V + e] * (double)beta[k];
            m[c] = acc;
            if (v_model) v_model[e] = acc;
        }
        for (int c = 0; c < 3; ++c)
            v[(size_t)c * V + i] = ((R[3 * c] * m[0] + R[3 * c + 1] * m[1]) + R[3 * c + 2] * m[2]) + (double)pose[3 + c];
    }
}

void orc_blend_albedo(int32_t V, int32_t n_alb, const float *alb_mean,
                      const float *b_alb, const float *delta, double *A) {
    for (size_t e = 0; e < (size_t)3 * V; ++e) {
        double acc = alb_mean[e];
        for (int k = 0; k < n_alb; ++k) acc = acc + (double)b_alb[(size_t)k * 3 * V + e] * (double)delta[k];
        A[e] = acc;
    }
}

void orc_vertex_normals(int32_t V, int32_t F, const int32_t *faces,
                        const double *pos, double *nrm) {
    /* sum in ascending face order: a plain loop over faces does exactly that */
    memset(nrm, 0, sizeof(double) * 3 * (size_t)V);
    for (int32_t f = 0; f < F; ++f) {
        int i0 = faces[3 * f], i1 = faces[3 * f + 1], i2 = faces[3 * f + 2];
        d3 v0 = dmk(pos[i0], pos[V + i0], pos[2 * V + i0]);
        d3 v1 = dmk(pos[i1], pos[V + i1], pos[2 * V + i1]);
        d3 v2 = dmk(pos[i2], pos[V + i2], pos[2 * V + i2]);
        d3 n = dcross(dsub(v1, v0), dsub(v2, v0));
        dacc(nrm, V, i0, n); dacc(nrm, V, i1, n); dacc(nrm, V, i2, n);
    }
    for (int32_t i = 0; i < V; ++i) {
        d3 n = dmk(nrm[i], nrm[V + i], nrm[2 * V + i]);
        double l = sqrt((n.x * n.x + n.y * n.y) + n.z * n.z);
        if (l > 0) { nrm[i] = n.x / l; nrm[V + i] = n.y / l; nrm[2 * V + i] = n.z / l; }
    }
}

/* --------------------------------------------------------------- edges -- */
typedef struct { int32_t a, b, f; } half_edge;
static int cmp_he(const void *p, const void *q) {
    const half_edge *x = p, *y = q;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return x->f < y->f ? -1 : (x->f > y->f);
}

int32_t orc_build_edges(int32_t V, int32_t F, const int32_t *faces, int32_t *out) {
    (void)V;
    half_edge *h = malloc(sizeof(half_edge) * 3 * (size_t)F);
    for (int32_t f = 0; f < F; ++f)
        for (int k = 0; k < 3; ++k) {
            int32_t a = faces[3 * f + k], b = faces[3 * f + (k + 1) % 3];
            half_edge e = {a < b ? a : b, a < b ? b : a, f};
            h[3 * f + k] = e;
        }
    qsort(h, 3 * (size_t)F, sizeof(half_edge), cmp_he);
    int32_t E = 0;
    for (size_t i = 0; i < 3 * (size_t)F;) {
        size_t j = i + 1;
        while (j < 3 * (size_t)F && h[j].a == h[i].a && h[j].b == h[i].b) ++j;
        if (j - i > 2) { free(h); return -1; }
        out[4 * E] = h[i].a; out[4 * E + 1] = h[i].b;
        out[4 * E + 2] = h[i].f; out[4 * E + 3] = (j - i == 2) ? h[i + 1].f : -1;
        ++E; i = j;
    }
    free(h);
    return E;
}

/* -------------------------------------------- ray/triangle (decisions) -- */
/* Moller-Trumbore in single precision, two-sided, inclusive barycentric
 * bounds, open t interval.  An accepted hit must also put o + t d inside the
 * triangle's bounding box widened by HIT_MARGIN: this makes "hit" a property
 * that any conservative acceleration structure reproduces exactly. */
static int ray_tri_f(f3 o, f3 d, f3 v0, f3 v1, f3 v2, float tmin, float tmax,
                     float *t_out, float *b1_out, float *b2_out, float *det_out) {
    f3 e1 = fsub(v1, v0), e2 = fsub(v2, v0);
    f3 pv = fcross(d, e2);
    float det = fdot(e1, pv);
    if (det == 0.0f) return 0;
    float inv = 1.0f / det;
    f3 tv = fsub(o, v0);
    float b1 = fdot(tv, pv) * inv;
    if (!(b1 >= 0.0f && b1 <= 1.0f)) return 0;
    f3 qv = fcross(tv, e1);
    float b2 = fdot(d, qv) * inv;
    if (!(b2 >= 0.0f && b1 + b2 <= 1.0f)) return 0;
    float t = fdot(e2, qv) * inv;
    if (!(t > tmin && t < tmax)) return 0;
    f3 P = {o.x + t * d.x, o.y + t * d.y, o.z + t * d.z};
    float lo, hi;
    lo = fminf(fminf(v0.x, v1.x), v2.x) - HIT_MARGIN; hi = fmaxf(fmaxf(v0.x, v1.x), v2.x) + HIT_MARGIN;
    if (!(P.x >= lo && P.x <= hi)) return 0;
    lo = fminf(fminf(v0.y, v1.y), v2.y) - HIT_MARGIN; hi = fmaxf(fmaxf(v0.y, v1.y), v2.y) + HIT_MARGIN;
    if (!(P.y >= lo && P.y <= hi)) return 0;
    lo = fminf(fminf(v0.z, v1.z), v2.z) - HIT_MARGIN; hi = fmaxf(fmaxf(v0.z, v1.z), v2.z) + HIT_MARGIN;
    if (!(P.z >= lo && P.z <= hi)) return 0;
    *t_out = t; *b1_out = b1; *b2_out = b2; *det_out = det;
    return 1;
}

int orc_ray_tri(const float o[3], const float d[3], const float v0[3],
                const float v1[3], const float v2[3], float tmin, float tmax,
                float *t, float *b1, float *b2, float *det) {
    f3 O = {o[0], o[1], o[2]}, D = {d[0], d[1], d[2]};
    f3 A = {v0[0], v0[1], v0[2]}, B = {v1[0], v1[1], v1[2]}, C = {v2[0], v2[1], v2[2]};
    return ray_tri_f(O, D, A, B, C, tmin, tmax, t, b1, b2, det);
}

/* ----------------------------------------------------- oracle's own BVH -- */
/* Top-down median split, up to 4 triangles per leaf, boxes padded by
 * BOX_PAD; traversed with a double-precision slab test.  Only an
 * accelerator: the hit definition above is what decides. */
typedef struct { double lo[3], hi[3]; int32_t left, right, first, count; } onode;
typedef struct { onode *n; int32_t *idx; int32_t nn; } obvh;

static const orc_scene *g_sort_scene;
static int g_sort_axis;
static double centroid_axis(const orc_scene *s, int f, int ax) {
    const int32_t *t = s->faces + 3 * f;
    return ((double)s->pos[ax * s->V + t[0]] + s->pos[ax * s->V + t[1]]) + s->pos[ax * s->V + t[2]];
}
static int cmp_cent(const void *p, const void *q) {
    int a = *(const int32_t *)p, b = *(const int32_t *)q;
    double ca = centroid_axis(g_sort_scene, a, g_sort_axis), cb = centroid_axis(g_sort_scene, b, g_sort_axis);
    if (ca != cb) return ca < cb ? -1 : 1;
    return a < b ? -1 : (a > b);
}

static int32_t bvh_build_rec(obvh *B, const orc_scene *s, int32_t first, int32_t count) {
    int32_t me = B->nn++;
    onode *n = &B->n[me];
    for (int a = 0; a < 3; ++a) { n->lo[a] = 1e300; n->hi[a] = -1e300; }
    double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
    for (int32_t i = first; i < first + count; ++i) {
        const int32_t *t = s->faces + 3 * B->idx[i];
        for (int a = 0; a < 3; ++a) {
            for (int k = 0; k < 3; ++k) {
                double v = s->pos[a * s->V + t[k]];
                if (v < n->lo[a]) n->lo[a] = v;
                if (v > n->hi[a]) n->hi[a] = v;
            }
            double c = centroid_axis(s, B->idx[i], a);
            if (c < clo[a]) clo[a] = c;
            if (c > chi[a]) chi[a] = c;
        }
    }
    for (int a = 0; a < 3; ++a) { n->lo[a] -= BOX_PAD; n->hi[a] += BOX_PAD; }
    n->first = first; n->count = count; n->left = n->right = -1;
    if (count <= 4) return me;
    int ax = 0;
    for (int a = 1; a < 3; ++a) if (chi[a] - clo[a] > chi[ax] - clo[ax]) ax = a;
    g_sort_scene = s; g_sort_axis = ax;
    qsort(B->idx + first, count, sizeof(int32_t), cmp_cent);
    int32_t half = count / 2;
    int32_t l = bvh_build_rec(B, s, first, half);
    int32_t r = bvh_build_rec(B, s, first + half, count - half);
    B->n[me].left = l; B->n[me].right = r; B->n[me].count = 0;
    return me;
}

static obvh *bvh_build(const orc_scene *s) {
    obvh *B = malloc(sizeof(obvh));
    B->n = malloc(sizeof(onode) * 2 * (size_t)(s->F + 1));
    B->idx = malloc(sizeof(int32_t) * (size_t)(s->F + 1));
    for (int32_t i = 0; i < s->F; ++i) B->idx[i] = i;
    B->nn = 0;
    if (s->F > 0) bvh_build_rec(B, s, 0, s->F);
    return B;
}
static void bvh_free(obvh *B) { if (B) { free(B->n); free(B->idx); free(B); } }

static int box_hit(const onode *n, f3 o, f3 d, double tmax) {
    double o3[3] = {o.x, o.y, o.z}, d3v[3] = {d.x, d.y, d.z};
    double t0 = 0.0, t1 = tmax * (1.0 + 1e-9) + 1e-12;
    for (int a = 0; a < 3; ++a) {
        if (d3v[a] == 0.0) {
            if (o3[a] < n->lo[a] || o3[a] > n->hi[a]) return 0;
            continue;
        }
        double ta = (n->lo[a] - o3[a]) / d3v[a], tb = (n->hi[a] - o3[a]) / d3v[a];
        if (ta > tb) { double x = ta; ta = tb; tb = x; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

/* closest: lexicographic (t, triangle index) */
static int32_t trace_closest(const orc_scene *s, const obvh *B, f3 o, f3 d,
                             float *t_out, float *b1o, float *b2o, float *deto) {
    int32_t best = -1;
    float bt = INFINITY, bb1 = 0, bb2 = 0, bdet = 0;
    if (!B) {
        for (int32_t f = 0; f < s->F; ++f) {
            const int32_t *tr = s->faces + 3 * f;
            float t, b1, b2, det;
            if (ray_tri_f(o, d, fpos(s, tr[0]), fpos(s, tr[1]), fpos(s, tr[2]), 0.0f, INFINITY, &t, &b1, &b2, &det)) {
                if (t < bt || (t == bt && f < best)) { bt = t; best = f; bb1 = b1; bb2 = b2; bdet = det; }
            }
        }
    } else if (B->nn > 0) {
        int32_t stack[128]; int sp = 0; stack[sp++] = 0;
        while (sp) {
            const onode *n = &B->n[stack[--sp]];
            if (!box_hit(n, o, d, best < 0 ? 1e30 : (double)bt)) continue;
            if (n->left < 0) {
                for (int32_t i = n->first; i < n->first + n->count; ++i) {
                    int32_t f = B->idx[i];
                    const int32_t *tr = s->faces + 3 * f;
                    float t, b1, b2, det;
                    if (ray_tri_f(o, d, fpos(s, tr[0]), fpos(s, tr[1]), fpos(s, tr[2]), 0.0f, INFINITY, &t, &b1, &b2, &det)) {
                        if (t < bt || (t == bt && f < best)) { bt = t; best = f; bb1 = b1; bb2 = b2; bdet = det; }
                    }
                }
            } else {
                stack[sp++] = n->left; stack[sp++] = n->right;
            }
        }
    }
    *t_out = bt; *b1o = bb1; *b2o = bb2; *deto = bdet;
    return best;
}

static int trace_any(const orc_scene *s, const obvh *B, f3 o, f3 d, int32_t skip) {
    float t, b1, b2, det;
    if (!B) {
        for (int32_t f = 0; f < s->F; ++f) {
            if (f == skip) continue;
            const int32_t *tr = s->faces + 3 * f;
            if (ray_tri_f(o, d, fpos(s, tr[0]), fpos(s, tr[1]), fpos(s, tr[2]), SHADOW_TMIN, SHADOW_TMAX, &t, &b1, &b2, &det))
                return 1;
        }
        return 0;
    }
    if (B->nn == 0) return 0;
    int32_t stack[128]; int sp = 0; stack[sp++] = 0;
    while (sp) {
        const onode *n = &B->n[stack[--sp]];
        if (!box_hit(n, o, d, 1.0)) continue;
        if (n->left < 0) {
            for (int32_t i = n->first; i < n->first + n->count; ++i) {
                int32_t f = B->idx[i];
                if (f == skip) continue;
                const int32_t *tr = s->faces + 3 * f;
                if (ray_tri_f(o, d, fpos(s, tr[0]), fpos(s, tr[1]), fpos(s, tr[2]), SHADOW_TMIN, SHADOW_TMAX, &t, &b1, &b2, &det))
                    return 1;
            }
        } else {
            stack[sp++] = n->left; stack[sp++] = n->right;
        }
    }
    return 0;
}

int32_t orc_closest_hit(const orc_scene *s, int use_bvh, const float o[3],
                        const float d[3], float *t, float *b1, float *b2, float *det) {
    obvh *B = use_bvh ? bvh_build(s) : NULL;
    f3 O = {o[0], o[1], o[2]}, D = {d[0], d[1], d[2]};
    int32_t r = trace_closest(s, B, O, D, t, b1, b2, det);
    bvh_free(B);
    return r;
}

int orc_any_hit(const orc_scene *s, int use_bvh, const float o[3], const float d[3], int32_t skip) {
    obvh *B = use_bvh ? bvh_build(s) : NULL;
    f3 O = {o[0], o[1], o[2]}, D = {d[0], d[1], d[2]};
    int r = trace_any(s, B, O, D, skip);
    bvh_free(B);
    return r;
}

/* ------------------------------------------------------ render context -- */
typedef struct {
    const orc_scene *s;
    obvh *bvh;
    float *nrm_f;      /* [3][V] vertex normals, single (decision input)     */
    double *nrm_d;     /* [3][V] vertex normals, double (value path)         */
    double *nrm_len;   /* [V] |sum of face normals| in the value path        */
    int32_t E;
    int32_t *edges;    /* [E][4]                                              */
    /* camera-silhouette sampling */
    uint64_t *pe_prefix; uint64_t pe_Q;
    /* shadow-boundary sampling: per light */
    uint64_t *se_prefix; uint64_t *se_Q;   /* [n][E], [n] */
} rctx;

static inline f3 light_c(const orc_scene *s, int j) { const float *g = s->light_geom + 12 * j; f3 r = {g[0], g[1], g[2]}; return r; }
static inline f3 light_e1(const orc_scene *s, int j) { const float *g = s->light_geom + 12 * j; f3 r = {g[3], g[4], g[5]}; return r; }
static inline f3 light_e2(const orc_scene *s, int j) { const float *g = s->light_geom + 12 * j; f3 r = {g[6], g[7], g[8]}; return r; }
static inline f3 light_n(const orc_scene *s, int j) { const float *g = s->light_geom + 12 * j; f3 r = {g[9], g[10], g[11]}; return r; }
static inline double light_area(const orc_scene *s, int j) {
    return dlen(dcross(d_of(light_e1(s, j)), d_of(light_e2(s, j))));
}

static inline f3 face_normal_f(const orc_scene *s, int32_t f) {
    const int32_t *t = s->faces + 3 * f;
    f3 v0 = fpos(s, t[0]);
    return fcross(fsub(fpos(s, t[1]), v0), fsub(fpos(s, t[2]), v0));
}

/* exclusive prefix of quantised weights; returns the total */
static uint64_t quantise_prefix(const float *w, int32_t n, uint64_t *prefix) {
    float wmax = 0.0f;
    for (int32_t i = 0; i < n; ++i) if (w[i] > wmax) wmax = w[i];
    uint64_t acc = 0;
    for (int32_t i = 0; i < n; ++i) {
        prefix[i] = acc;
        if (w[i] > 0.0f && wmax > 0.0f) acc += 1u + (uint32_t)floorf((w[i] / wmax) * QSCALE);
    }
    return acc;
}

/* largest i with prefix[i] <= target (prefix non-decreasing, prefix[0] = 0) */
static int32_t cdf_pick(const uint64_t *prefix, int32_t n, uint64_t target) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo + 1) / 2;
        if (prefix[mid] <= target) lo = mid; else hi = mid - 1;
    }
    return lo;
}
static inline uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}
static inline uint64_t edge_weight(const uint64_t *prefix, int32_t n, uint64_t Q, int32_t i) {
    return (i + 1 < n ? prefix[i + 1] : Q) - prefix[i];
}

/* screen projection (single): x' = W/2 + (x/-z)/ps, y' = H/2 - (y/-z)/ps */
static int project_f(const orc_scene *s, f3 x, float *sx, float *sy) {
    f3 c = {s->cam[0], s->cam[1], s->cam[2]};
    f3 r = fsub(x, c);
    if (!(r.z < 0.0f)) return 0;
    float nz = -r.z;
    *sx = 0.5f * (float)s->W + (r.x / nz) / s->pix_scale;
    *sy = 0.5f * (float)s->H - (r.y / nz) / s->pix_scale;
    return 1;
}

static void build_edge_tables(rctx *C) {
    const orc_scene *s = C->s;
    int32_t *tmp = malloc(sizeof(int32_t) * 4 * 3 * (size_t)(s->F + 1));
    C->E = orc_build_edges(s->V, s->F, s->faces, tmp);
    C->edges = tmp;
    int32_t E = C->E > 0 ? C->E : 0;
    float *w = malloc(sizeof(float) * (size_t)(E + 1));
    f3 cam = {s->cam[0], s->cam[1], s->cam[2]};
    /* camera silhouette: boundary edges, or faces on opposite sides */
    for (int32_t e = 0; e < E; ++e) {
        const int32_t *ed = C->edges + 4 * e;
        int sil = 1;
        if (ed[3] >= 0) {
            float s1 = fdot(face_normal_f(s, ed[2]), fsub(cam, fpos(s, s->faces[3 * ed[2]])));
            float s2 = fdot(face_normal_f(s, ed[3]), fsub(cam, fpos(s, s->faces[3 * ed[3]])));
            sil = (s1 > 0.0f) != (s2 > 0.0f);
        }
        float ax, ay, bx, by;
        w[e] = 0.0f;
        if (sil && project_f(s, fpos(s, ed[0]), &ax, &ay) && project_f(s, fpos(s, ed[1]), &bx, &by)) {
            float dx = bx - ax, dy = by - ay;
            w[e] = sqrtf(dx * dx + dy * dy);
        }
    }
    C->pe_prefix = malloc(sizeof(uint64_t) * (size_t)(E + 1));
    C->pe_Q = quantise_prefix(w, E, C->pe_prefix);
    /* shadow-boundary candidates per light */
    int n = s->n_lights;
    C->se_prefix = malloc(sizeof(uint64_t) * (size_t)n * (E + 1));
    C->se_Q = malloc(sizeof(uint64_t) * (size_t)n);
    for (int j = 0; j < n; ++j) {
        f3 c = light_c(s, j), e1 = light_e1(s, j), e2 = light_e2(s, j);
        f3 corner[4];
        for (int k = 0; k < 4; ++k) {
            float s1 = (k & 1) ? 0.5f : -0.5f, s2 = (k & 2) ? 0.5f : -0.5f;
            corner[k].x = (c.x + s1 * e1.x) + s2 * e2.x;
            corner[k].y = (c.y + s1 * e1.y) + s2 * e2.y;
            corner[k].z = (c.z + s1 * e1.z) + s2 * e2.z;
        }
        for (int32_t e = 0; e < E; ++e) {
            const int32_t *ed = C->edges + 4 * e;
            int cand = 1;
            if (ed[3] >= 0) {
                f3 n1 = face_normal_f(s, ed[2]), n2 = face_normal_f(s, ed[3]);
                f3 o1 = fpos(s, s->faces[3 * ed[2]]), o2 = fpos(s, s->faces[3 * ed[3]]);
                int pos = 0, neg = 0;
                for (int k = 0; k < 4; ++k) {
                    int g1 = fdot(n1, fsub(corner[k], o1)) > 0.0f;
                    int g2 = fdot(n2, fsub(corner[k], o2)) > 0.0f;
                    pos += g1 + g2; neg += 2 - g1 - g2;
                }
                cand = pos > 0 && neg > 0;
            }
            w[e] = 0.0f;
            if (cand) {
                f3 ab = fsub(fpos(s, ed[1]), fpos(s, ed[0]));
                w[e] = sqrtf(fdot(ab, ab));
            }
        }
        C->se_Q[j] = quantise_prefix(w, E, C->se_prefix + (size_t)j * (E + 1));
    }
    free(w);
}

static int rctx_init(rctx *C, const orc_scene *s, int want_edges) {
    memset(C, 0, sizeof(*C));
    if (s->n_lights > MAXL || s->n_lights < 0 || s->W <= 0 || s->H <= 0) return -1;
    C->s = s;
    C->bvh = bvh_build(s);
    size_t V = (size_t)s->V;
    double *tmp = malloc(sizeof(double) * 3 * V), *tn = malloc(sizeof(double) * 3 * V);
    for (size_t i = 0; i < 3 * V; ++i) tmp[i] = (double)s->pos[i];
    orc_vertex_normals(s->V, s->F, s->faces, tmp, tn);
    C->nrm_f = malloc(sizeof(float) * 3 * V);
    for (size_t i = 0; i < 3 * V; ++i) C->nrm_f[i] = (float)tn[i];
    free(tmp); free(tn);
    /* value-path normals from the double positions, keeping |sum| for the chain */
    C->nrm_d = calloc(3 * V, sizeof(double));
    C->nrm_len = calloc(V, sizeof(double));
    for (int32_t f = 0; f < s->F; ++f) {
        const int32_t *t = s->faces + 3 * f;
        d3 v0 = dpos(s, t[0]);
        d3 n = dcross(dsub(dpos(s, t[1]), v0), dsub(dpos(s, t[2]), v0));
        for (int k = 0; k < 3; ++k) dacc(C->nrm_d, s->V, t[k], n);
    }
    for (size_t i = 0; i < V; ++i) {
        d3 n = dmk(C->nrm_d[i], C->nrm_d[V + i], C->nrm_d[2 * V + i]);
        double l = dlen(n);
        C->nrm_len[i] = l;
        if (l > 0) { C->nrm_d[i] = n.x / l; C->nrm_d[V + i] = n.y / l; C->nrm_d[2 * V + i] = n.z / l; }
    }
    if (want_edges) build_edge_tables(C);
    return 0;
}

static void rctx_free(rctx *C) {
    bvh_free(C->bvh);
    free(C->nrm_f); free(C->nrm_d); free(C->nrm_len);
    free(C->edges); free(C->pe_prefix); free(C->se_prefix); free(C->se_Q);
}

/* ------------------------------------------------- decisions per sample -- */
typedef struct {
    int32_t tri;            /* -1: miss */
    int front;              /* camera sees the side e1 x e2 points to */
    int spec_on;            /* viewer above the interpolated normal   */
    uint64_t vis;           /* bit j: light sample j lit (horizon and shadow) */
    float b1, b2;           /* single-precision barycentrics          */
    f3 p;                   /* single-precision shading point         */
    f3 nu;                  /* interpolated vertex normal (unflipped) */
    f3 wod;                 /* unit direction to the camera           */
    int tex_ix, tex_iy;     /* bilinear texel cell of the specular map */
    f3 y[MAXL];             /* light sample points                    */
    uint64_t cs_on, cl_on;  /* bit j: light sample j above the shading
                               normal / in front of the emitter        */
    unsigned char gsel[MAXL]; /* V-cavity branch: 0 G=1, 1 G1, 2 G2   */
} sdec;

/* Branches of the shading whose value is continuous but whose slope jumps
 * (the clamps of cos_s and cos_l, the min of the V-cavity term) are taken
 * as single-precision decisions too, from the decision values of the
 * sample, so that value path and adjoint follow the same branch on every
 * implementation.  The V-cavity comparisons are G1, G2 >= 1 and G1 <= G2
 * written with unnormalised dot products (all positive factors cancel). */
static void light_branch(const sdec *D, f3 nj, f3 y, int *cs, int *cl, int *gs) {
    f3 r = fsub(y, D->p);
    f3 nn = D->nu;
    if (!D->front) { nn.x = -nn.x; nn.y = -nn.y; nn.z = -nn.z; }
    *cs = fdot(nn, r) > 0.0f;
    *cl = fdot(nj, r) < 0.0f;
    *gs = 0;
    if (D->spec_on && *cs) {
        float lr = sqrtf(fdot(r, r));
        f3 wi = {r.x / lr, r.y / lr, r.z / lr};
        f3 hs = {wi.x + D->wod.x, wi.y + D->wod.y, wi.z + D->wod.z};
        float a_s = fdot(nn, wi), a_o = fdot(nn, D->wod);
        float nh = fdot(nn, hs), oh2 = fdot(D->wod, hs), n2 = fdot(D->nu, D->nu);
        float rhs = oh2 * n2;
        float g1 = (2.0f * nh) * a_o, g2 = (2.0f * nh) * a_s;
        if (g1 >= rhs && g2 >= rhs) *gs = 0;
        else if (a_o <= a_s) *gs = 1;
        else *gs = 2;
    }
}

static inline f3 light_point(const orc_scene *s, int j, float u, float v) {
    f3 c = light_c(s, j), e1 = light_e1(s, j), e2 = light_e2(s, j);
    float a = u - 0.5f, b = v - 0.5f;
    f3 y = {(c.x + a * e1.x) + b * e2.x, (c.y + a * e1.y) + b * e2.y, (c.z + a * e1.z) + b * e2.z};
    return y;
}

static inline f3 camera_dir(const orc_scene *s, float qx, float qy) {
    f3 d = {(qx - 0.5f * (float)s->W) * s->pix_scale, (0.5f * (float)s->H - qy) * s->pix_scale, -1.0f};
    return d;
}

/* Decide everything discrete for a camera ray through screen point (qx,qy)
 * with light uniforms lu[2j], lu[2j+1]. */
static void decide(const rctx *C, float qx, float qy, const float *lu, sdec *D, orc_counts *cnt) {
    const orc_scene *s = C->s;
    f3 o = {s->cam[0], s->cam[1], s->cam[2]};
    f3 d = camera_dir(s, qx, qy);
    float t, b1, b2, det;
    if (cnt) cnt->camera++;
    D->tri = trace_closest(s, C->bvh, o, d, &t, &b1, &b2, &det);
    D->vis = 0;
    if (D->tri < 0) return;
    const int32_t *tr = s->faces + 3 * D->tri;
    f3 v0 = fpos(s, tr[0]), v1 = fpos(s, tr[1]), v2 = fpos(s, tr[2]);
    D->b1 = b1; D->b2 = b2;
    D->front = det > 0.0f;
    float b0 = (1.0f - b1) - b2;
    f3 p = {(b0 * v0.x + b1 * v1.x) + b2 * v2.x, (b0 * v0.y + b1 * v1.y) + b2 * v2.y,
            (b0 * v0.z + b1 * v1.z) + b2 * v2.z};
    D->p = p;
    /* specular lobe: viewer on the positive side of the (flipped) interpolated normal */
    const float *N = C->nrm_f; int V = s->V;
    f3 nu;
    nu.x = (b0 * N[tr[0]] + b1 * N[tr[1]]) + b2 * N[tr[2]];
    nu.y = (b0 * N[V + tr[0]] + b1 * N[V + tr[1]]) + b2 * N[V + tr[2]];
    nu.z = (b0 * N[2 * V + tr[0]] + b1 * N[2 * V + tr[1]]) + b2 * N[2 * V + tr[2]];
    float co = fdot(nu, fsub(o, p));
    D->spec_on = D->front ? co > 0.0f : co < 0.0f;
    D->nu = nu;
    f3 c = fsub(o, p);
    float lc = sqrtf(fdot(c, c));
    D->wod.x = c.x / lc; D->wod.y = c.y / lc; D->wod.z = c.z / lc;
    /* texel cell: texel centres at (i + 1/2)/res */
    float ux = (b0 * s->uv[tr[0]] + b1 * s->uv[tr[1]]) + b2 * s->uv[tr[2]];
    float uy = (b0 * s->uv[V + tr[0]] + b1 * s->uv[V + tr[1]]) + b2 * s->uv[V + tr[2]];
    D->tex_ix = (int)floorf((float)s->spec_res * ux - 0.5f);
    D->tex_iy = (int)floorf((float)s->spec_res * uy - 0.5f);
    D->cs_on = D->cl_on = 0;
    f3 ng = fcross(fsub(v1, v0), fsub(v2, v0));
    for (int j = 0; j < s->n_lights; ++j) {
        f3 y = light_point(s, j, lu[2 * j], lu[2 * j + 1]);
        D->y[j] = y;
        int cs, cl, gs;
        light_branch(D, light_n(s, j), y, &cs, &cl, &gs);
        D->cs_on |= (uint64_t)cs << j;
        D->cl_on |= (uint64_t)cl << j;
        D->gsel[j] = (unsigned char)gs;
        f3 r = fsub(y, p);
        float hz = fdot(ng, r);
        int above = D->front ? hz > 0.0f : hz < 0.0f;
        if (!above) continue;
        if (cnt) cnt->shadow++;
        if (!trace_any(s, C->bvh, p, r, D->tri)) D->vis |= (uint64_t)1 << j;
    }
}

/* ------------------------------------------------------- value path ----- */
/* per-sample geometry in double for the hit triangle */
typedef struct {
    int32_t i[3];
    d3 v[3], n[3];
    double b[3];        /* b0, b1, b2 */
    d3 p, nu, ns, wo;
    double nlen, olen, sgn, cos_o;
    double A[3];        /* interpolated albedo */
    double uvx, uvy, ks;
    /* bilinear texel footprint */
    int tex[4]; double tw[4]; double dks_du, dks_dv;
    d3 pv, e1xd;        /* for the barycentric chain */
    double det;
} sgeo;

static void geo_eval(const rctx *C, f3 of, f3 df, const sdec *D, sgeo *G) {
    const orc_scene *s = C->s;
    int V = s->V;
    const int32_t *tr = s->faces + 3 * D->tri;
    for (int k = 0; k < 3; ++k) {
        G->i[k] = tr[k];
        G->v[k] = dpos(s, tr[k]);
        G->n[k] = dmk(C->nrm_d[tr[k]], C->nrm_d[V + tr[k]], C->nrm_d[2 * V + tr[k]]);
    }
    d3 o = d_of(of), d = d_of(df);
    d3 e1 = dsub(G->v[1], G->v[0]), e2 = dsub(G->v[2], G->v[0]);
    d3 pv = dcross(d, e2);
    double det = ddot(e1, pv);
    d3 tv = dsub(o, G->v[0]);
    double b1 = ddot(tv, pv) / det;
    d3 qv = dcross(tv, e1);
    double b2 = ddot(d, qv) / det;
    G->b[0] = 1.0 - b1 - b2; G->b[1] = b1; G->b[2] = b2;
    G->pv = pv; G->e1xd = dcross(e1, d); G->det = det;
    G->p = dadd(dadd(dscl(G->v[0], G->b[0]), dscl(G->v[1], b1)), dscl(G->v[2], b2));
    G->nu = dadd(dadd(dscl(G->n[0], G->b[0]), dscl(G->n[1], b1)), dscl(G->n[2], b2));
    G->nlen = dlen(G->nu);
    G->sgn = D->front ? 1.0 : -1.0;
    G->ns = dscl(G->nu, G->sgn / G->nlen);
    for (int c = 0; c < 3; ++c)
        G->A[c] = G->b[0] * s->alb[c * V + tr[0]] + b1 * s->alb[c * V + tr[1]] + b2 * s->alb[c * V + tr[2]];
    G->uvx = G->b[0] * s->uv[tr[0]] + b1 * s->uv[tr[1]] + b2 * s->uv[tr[2]];
    G->uvy = G->b[0] * s->uv[V + tr[0]] + b1 * s->uv[V + tr[1]] + b2 * s->uv[V + tr[2]];
    /* bilinear, texel centres at (i+0.5)/res, clamp to edge */
    int R = s->spec_res;
    /* the cell is a decision (its slope jumps at texel centres); the
       weights are the value path's, linear beyond the cell if need be */
    double x = R * G->uvx - 0.5, y = R * G->uvy - 0.5;
    int ix0 = D->tex_ix, iy0 = D->tex_iy;
    double fx = x - ix0, fy = y - iy0;
    int ix[2] = {ix0, ix0 + 1}, iy[2] = {iy0, iy0 + 1};
    for (int k = 0; k < 2; ++k) {
        ix[k] = ix[k] < 0 ? 0 : (ix[k] > R - 1 ? R - 1 : ix[k]);
        iy[k] = iy[k] < 0 ? 0 : (iy[k] > R - 1 ? R - 1 : iy[k]);
    }
    G->tex[0] = iy[0] * R + ix[0]; G->tw[0] = (1 - fx) * (1 - fy);
    G->tex[1] = iy[0] * R + ix[1]; G->tw[1] = fx * (1 - fy);
    G->tex[2] = iy[1] * R + ix[0]; G->tw[2] = (1 - fx) * fy;
    G->tex[3] = iy[1] * R + ix[1]; G->tw[3] = fx * fy;
    const double *T = s->spec;
    G->ks = G->tw[0] * T[G->tex[0]] + G->tw[1] * T[G->tex[1]] + G->tw[2] * T[G->tex[2]] + G->tw[3] * T[G->tex[3]];
    G->dks_du = R * ((1 - fy) * (T[G->tex[1]] - T[G->tex[0]]) + fy * (T[G->tex[3]] - T[G->tex[2]]));
    G->dks_dv = R * ((1 - fx) * (T[G->tex[2]] - T[G->tex[0]]) + fx * (T[G->tex[3]] - T[G->tex[1]]));
    d3 wv = dsub(o, G->p);
    G->olen = dlen(wv);
    G->wo = dscl(wv, 1.0 / G->olen);
    G->cos_o = ddot(G->ns, G->wo);
}

/* One light's shaded contribution at the sample, and (optionally) its
 * adjoint.  Radiance c = l (A/pi cos_s + S) cos_l area / d^2 with
 * S = f_s cos_s = ks D G / (4 cos_o) (Beckmann D, V-cavity G, F = 1). */
typedef struct {
    d3 gp, gns, gwo;     /* adjoints w.r.t. p, n_s, w_o  */
    double gA[3], gks;   /* adjoints w.r.t. albedo, ks   */
    double gl[3];        /* adjoint w.r.t. l_j           */
} ladj;

static void shade_light(const rctx *C, const sgeo *G, int spec_on, int cs_on, int cl_on, int gsel_in,
                        int j, d3 y, const double *w /* RGB weights or NULL */, double out[3], ladj *adj) {
    const orc_scene *s = C->s;
    const double *l = s->light_rgb + 3 * j;
    d3 nj = d_of(light_n(s, j));
    double area = light_area(s, j);
    d3 r = dsub(y, G->p);
    double d2 = ddot(r, r), dist = sqrt(d2);
    d3 wi = dscl(r, 1.0 / dist);
    /* clamps and the V-cavity min follow the sample's decisions */
    double cl_raw = -ddot(nj, wi), cos_l = cl_on ? cl_raw : 0;
    double cs_raw = ddot(G->ns, wi), cos_s = cs_on ? cs_raw : 0;
    double g = cos_l * area / d2;
    double S = 0, D = 0, Gv = 0, ch = 0, oh = 0, lh = 0;
    int gsel = gsel_in;      /* 0: G = 1, 1: G1, 2: G2 */
    d3 h = dmk(0, 0, 0);
    int spec = spec_on && cs_on;
    if (spec) {
        d3 hv = dadd(wi, G->wo);
        lh = dlen(hv);
        h = dscl(hv, 1.0 / lh);
        ch = ddot(G->ns, h);
        oh = ddot(G->wo, h);
        double m2 = BECKMANN_M * BECKMANN_M, c2 = ch * ch;
        D = exp(-(1.0 - c2) / (c2 * m2)) / (PI * m2 * c2 * c2);
        double G1 = 2.0 * ch * G->cos_o / oh, G2 = 2.0 * ch * cos_s / oh;
        Gv = gsel == 0 ? 1.0 : (gsel == 1 ? G1 : G2);
        S = G->ks * D * Gv / (4.0 * G->cos_o);
    }
    for (int c = 0; c < 3; ++c) out[c] = l[c] * (G->A[c] / PI * cos_s + S) * g;
    if (!adj) return;
    /* reverse mode */
    double Ld = 0, Lw = 0;
    for (int c = 0; c < 3; ++c) {
        adj->gl[c] = w[c] * (G->A[c] / PI * cos_s + S) * g;
        adj->gA[c] = w[c] * l[c] * cos_s * g / PI;
        Ld += w[c] * l[c] * G->A[c] / PI;
        Lw += w[c] * l[c];
    }
    double g_cos_s = Ld * g;
    double g_S = Lw * g;
    double g_g = Ld * cos_s + Lw * S;
    adj->gks = spec ? g_S * D * Gv / (4.0 * G->cos_o) : 0.0;
    double g_cos_l = g_g * area / d2;
    double g_d2 = -g_g * g / d2;
    d3 g_wi = dmk(0, 0, 0), g_ns = dmk(0, 0, 0), g_wo = dmk(0, 0, 0);
    double g_cos_o = 0;
    if (spec) {
        /* dS/dD * dD/dch = S (2/(m^2 ch^3) - 4/ch), written without S/D */
        double g_G = g_S * G->ks * D / (4.0 * G->cos_o);
        g_cos_o += -g_S * S / G->cos_o;
        double m2 = BECKMANN_M * BECKMANN_M;
        double g_ch = g_S * S * (2.0 / (m2 * ch * ch * ch) - 4.0 / ch);
        double g_oh = 0;
        if (gsel == 1) {
            g_ch += g_G * 2.0 * G->cos_o / oh;
            g_cos_o += g_G * 2.0 * ch / oh;
            g_oh += -g_G * Gv / oh;
        } else if (gsel == 2) {
            g_ch += g_G * 2.0 * cos_s / oh;
            g_cos_s += g_G * 2.0 * ch / oh;
            g_oh += -g_G * Gv / oh;
        }
        /* ch = ns.h, oh = wo.h */
        g_ns = dadd(g_ns, dscl(h, g_ch));
        g_wo = dadd(g_wo, dscl(h, g_oh));
        d3 g_h = dadd(dscl(G->ns, g_ch), dscl(G->wo, g_oh));
        d3 g_hv = dnorm_adj(g_h, h, lh);
        g_wi = dadd(g_wi, g_hv);
        g_wo = dadd(g_wo, g_hv);
    }
    /* cos_o = ns.wo */
    g_ns = dadd(g_ns, dscl(G->wo, g_cos_o));
    g_wo = dadd(g_wo, dscl(G->ns, g_cos_o));
    /* clamps */
    double g_cs_raw = cs_on ? g_cos_s : 0;
    double g_cl_raw = cl_on ? g_cos_l : 0;
    g_ns = dadd(g_ns, dscl(wi, g_cs_raw));
    g_wi = dadd(g_wi, dscl(G->ns, g_cs_raw));
    g_wi = dadd(g_wi, dscl(nj, -g_cl_raw));
    /* wi = r/|r|, d2 = r.r, r = y - p */
    d3 g_r = dadd(dnorm_adj(g_wi, wi, dist), dscl(r, 2.0 * g_d2));
    adj->gp = dscl(g_r, -1.0);
    adj->gns = g_ns;
    adj->gwo = g_wo;
}

/* Full radiance of one sample given its decisions (sum over lit lights). */
static void sample_value(const rctx *C, f3 o, f3 d, const sdec *D, double out[3]) {
    out[0] = out[1] = out[2] = 0;
    if (D->tri < 0) return;
    sgeo G;
    geo_eval(C, o, d, D, &G);
    for (int j = 0; j < C->s->n_lights; ++j) {
        if (!((D->vis >> j) & 1)) continue;
        double c[3];
        shade_light(C, &G, D->spec_on, (D->cs_on >> j) & 1, (D->cl_on >> j) & 1, D->gsel[j], j,
                    d_of(D->y[j]), NULL, c, NULL);
        out[0] += c[0]; out[1] += c[1]; out[2] += c[2];
    }
}

/* Auxiliary buffers of one camera sample, for a denoiser: the first hit's
 * interpolated albedo, its shading normal turned toward the camera, and its
 * distance from the camera (all zero on a miss), added to acc[7].  The hit is
 * the estimator's own closest-hit decision; the values are the value path's
 * (double, barycentrics re-solved). */
static void sample_aov(const rctx *C, f3 o, f3 d, double acc[7]) {
    float t, b1, b2, det;
    sdec D;
    D.tri = trace_closest(C->s, C->bvh, o, d, &t, &b1, &b2, &det);
    if (D.tri < 0) return;
    D.front = det > 0.0f;
    D.b1 = b1; D.b2 = b2;
    D.tex_ix = D.tex_iy = 0;      /* texel cell: not used by the buffers */
    sgeo G;
    geo_eval(C, o, d, &D, &G);
    acc[0] += G.A[0]; acc[1] += G.A[1]; acc[2] += G.A[2];
    acc[3] += G.ns.x; acc[4] += G.ns.y; acc[5] += G.ns.z;
    acc[6] += G.olen;
}

/* ------------------------------------------------ thread-parallel driver -- */
typedef struct {
    double *d_light, *d_spec, *d_pos, *d_nrm, *d_alb, *d_pos_pe, *d_pos_se;
} gbuf;

typedef struct {
    rctx *C;
    uint64_t seed;
    int32_t spp;
    int64_t s0, s1;             /* camera sample range, or edge sample range */
    double *image;              /* forward: [H][W][3] accumulated (disjoint pixels) */
    const int32_t *rec_in;      /* frozen decisions */
    int32_t *rec_out;
    const double *dLdI;
    int32_t flags;
    gbuf g;
    orc_counts cnt;
    int mode;                   /* 0 render, 1 record, 2 frozen render, 3 backward, 4 frozen backward, 5 primary edges */
    const int32_t *pix; double *pix_out;
} job;

static void gbuf_alloc(gbuf *g, int V, int nl, int res) {
    g->d_light = calloc((size_t)3 * nl, sizeof(double));
    g->d_spec = calloc((size_t)res * res, sizeof(double));
    g->d_pos = calloc((size_t)3 * V, sizeof(double));
    g->d_nrm = calloc((size_t)3 * V, sizeof(double));
    g->d_alb = calloc((size_t)3 * V, sizeof(double));
    g->d_pos_pe = calloc((size_t)3 * V, sizeof(double));
    g->d_pos_se = calloc((size_t)3 * V, sizeof(double));
}
static void gbuf_free(gbuf *g) {
    free(g->d_light); free(g->d_spec); free(g->d_pos); free(g->d_nrm);
    free(g->d_alb); free(g->d_pos_pe); free(g->d_pos_se);
}

/* decode a record into decisions (light points regenerated from the RNG) */
static void rec_to_dec(const rctx *C, const int32_t *rec, const float *lu, sdec *D) {
    D->tri = rec[0];
    D->front = rec[1] & 1;
    D->spec_on = (rec[1] >> 1) & 1;
    D->vis = (uint32_t)rec[2];
    D->cs_on = (uint32_t)rec[3];
    D->cl_on = (uint32_t)rec[4];
    D->tex_ix = rec[7];
    D->tex_iy = rec[8];
    for (int j = 0; j < C->s->n_lights; ++j) {
        D->y[j] = light_point(C->s, j, lu[2 * j], lu[2 * j + 1]);
        D->gsel[j] = (unsigned char)(((uint32_t)rec[5 + j / 16] >> (2 * (j % 16))) & 3u);
    }
}

/* Chain p (ray fixed) and barycentric adjoints into the hit triangle's
 * vertices.  p = sum b_k v_k with (b1, b2) fixed by v0 + b1 e1 + b2 e2 = o + t d. */
static void chain_hit(const sgeo *G, d3 gp, double gb[3], double *d_pos, int V) {
    for (int k = 0; k < 3; ++k) {
        dacc(d_pos, V, G->i[k], dscl(gp, G->b[k]));
        gb[k] += ddot(G->v[k], gp);
    }
    double g1 = gb[1] - gb[0], g2 = gb[2] - gb[0];
    d3 z = dscl(dadd(dscl(G->pv, g1), dscl(G->e1xd, g2)), -1.0 / G->det);
    for (int k = 0; k < 3; ++k) dacc(d_pos, V, G->i[k], dscl(z, G->b[k]));
}

/* interior adjoint of one camera sample */
static void sample_adjoint(const rctx *C, f3 o, f3 d, const sdec *D, const double *w, gbuf *g) {
    const orc_scene *s = C->s;
    int V = s->V;
    sgeo G;
    geo_eval(C, o, d, D, &G);
    d3 gp = dmk(0, 0, 0), gns = dmk(0, 0, 0), gwo = dmk(0, 0, 0);
    double gA[3] = {0, 0, 0}, gks = 0;
    for (int j = 0; j < s->n_lights; ++j) {
        if (!((D->vis >> j) & 1)) continue;
        double c[3];
        ladj a;
        shade_light(C, &G, D->spec_on, (D->cs_on >> j) & 1, (D->cl_on >> j) & 1, D->gsel[j], j,
                    d_of(D->y[j]), w, c, &a);
        for (int k = 0; k < 3; ++k) { g->d_light[3 * j + k] += a.gl[k]; gA[k] += a.gA[k]; }
        gks += a.gks;
        gp = dadd(gp, a.gp); gns = dadd(gns, a.gns); gwo = dadd(gwo, a.gwo);
    }
    double gb[3] = {0, 0, 0};
    /* ks(uv): texels and uv */
    for (int k = 0; k < 4; ++k) g->d_spec[G.tex[k]] += gks * G.tw[k];
    double guvx = gks * G.dks_du, guvy = gks * G.dks_dv;
    for (int k = 0; k < 3; ++k) {
        int vi = G.i[k];
        gb[k] += guvx * s->uv[vi] + guvy * s->uv[V + vi];
        for (int c = 0; c < 3; ++c) {
            g->d_alb[c * V + vi] += G.b[k] * gA[c];
            gb[k] += gA[c] * s->alb[c * V + vi];
        }
    }
    /* wo = (o - p)/|o - p| */
    gp = dsub(gp, dnorm_adj(gwo, G.wo, G.olen));
    /* ns = sgn nu/|nu|, nu = sum b_k n_k */
    d3 nt = dscl(G.nu, 1.0 / G.nlen);
    d3 gnu = dnorm_adj(dscl(gns, G.sgn), nt, G.nlen);
    for (int k = 0; k < 3; ++k) {
        dacc(g->d_nrm, V, G.i[k], dscl(gnu, G.b[k]));
        gb[k] += ddot(G.n[k], gnu);
    }
    chain_hit(&G, gp, gb, g->d_pos, V);
}

/* Shadow-boundary term for camera sample sidx at shading point D (secondary
 * edges).  Accumulates into g->d_pos_se. */
static void sample_secondary(const rctx *C, uint64_t seed, int64_t sidx, f3 o, f3 d,
                             const sdec *D, const double *w, gbuf *g, orc_counts *cnt) {
    const orc_scene *s = C->s;
    int V = s->V, E = C->E;
    sgeo G;
    int geo_done = 0;
    const int32_t *tr = s->faces + 3 * D->tri;
    f3 v0 = fpos(s, tr[0]);
    f3 ngf = fcross(fsub(fpos(s, tr[1]), v0), fsub(fpos(s, tr[2]), v0));
    f3 p = D->p;
    for (int j = 0; j < s->n_lights; ++j) {
        uint64_t Q = C->se_Q[j];
        if (Q == 0) continue;
        uint32_t wds[4];
        orc_philox((uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)sidx, (uint32_t)j, 1, 0, wds);
        const uint64_t *pre = C->se_prefix + (size_t)j * (E + 1);
        uint64_t target = mulhi64(((uint64_t)wds[1] << 32) | wds[0], Q);
        int32_t e = cdf_pick(pre, E, target);
        const int32_t *ed = C->edges + 4 * e;
        if (ed[2] == D->tri || ed[3] == D->tri) continue;
        if (ed[3] >= 0) {
            float s1 = fdot(face_normal_f(s, ed[2]), fsub(p, fpos(s, s->faces[3 * ed[2]])));
            float s2 = fdot(face_normal_f(s, ed[3]), fsub(p, fpos(s, s->faces[3 * ed[3]])));
            if ((s1 > 0.0f) == (s2 > 0.0f)) continue;
        }
        float tu = u01(wds[2]);
        f3 a = fpos(s, ed[0]), b = fpos(s, ed[1]);
        f3 sp = {a.x + tu * (b.x - a.x), a.y + tu * (b.y - a.y), a.z + tu * (b.z - a.z)};
        f3 nj = light_n(s, j), cj = light_c(s, j);
        float den = fdot(nj, fsub(sp, p));
        if (den == 0.0f) continue;
        float lam = fdot(nj, fsub(cj, p)) / den;
        if (!(lam > 1.0f)) continue;
        f3 y = {p.x + lam * (sp.x - p.x), p.y + lam * (sp.y - p.y), p.z + lam * (sp.z - p.z)};
        f3 e1 = light_e1(s, j), e2 = light_e2(s, j);
        f3 ql = fsub(y, cj);
        if (!(fabsf(fdot(ql, e1)) <= 0.5f * fdot(e1, e1) && fabsf(fdot(ql, e2)) <= 0.5f * fdot(e2, e2))) continue;
        float hz = fdot(ngf, fsub(y, p));
        if (!(D->front ? hz > 0.0f : hz < 0.0f)) continue;
        f3 m = fcross(fsub(a, p), fsub(b, p));
        float mn = fdot(m, nj);
        f3 mp = {m.x - mn * nj.x, m.y - mn * nj.y, m.z - mn * nj.z};
        float lm = sqrtf(fdot(mp, mp));
        if (lm == 0.0f) continue;
        f3 un = {mp.x / lm, mp.y / lm, mp.z / lm};
        f3 yp = {y.x + EDGE_OFF_M * un.x, y.y + EDGE_OFF_M * un.y, y.z + EDGE_OFF_M * un.z};
        f3 ym = {y.x - EDGE_OFF_M * un.x, y.y - EDGE_OFF_M * un.y, y.z - EDGE_OFF_M * un.z};
        if (cnt) cnt->edge_secondary += 2;
        int vp = !trace_any(s, C->bvh, p, fsub(yp, p), D->tri);
        int vm = !trace_any(s, C->bvh, p, fsub(ym, p), D->tri);
        if (vp == vm) continue;
        /* value path */
        if (!geo_done) { geo_eval(C, o, d, D, &G); geo_done = 1; }
        d3 yd = d_of(y);
        double hc[3];
        int cs, cl, gs;
        light_branch(D, nj, y, &cs, &cl, &gs);
        shade_light(C, &G, D->spec_on, cs, cl, gs, j, yd, NULL, hc, NULL);
        /* hc includes the light area factor; the boundary integral is per unit area */
        double area = light_area(s, j);
        double hw = (w[0] * hc[0] + w[1] * hc[1] + w[2] * hc[2]) / area;
        d3 A = dpos(s, ed[0]), B = dpos(s, ed[1]), P = G.p, N = d_of(nj);
        d3 pa = dsub(A, P), pb = dsub(B, P), py = dsub(yd, P);
        d3 md = dcross(pa, pb);
        d3 mpar = dsub(md, dscl(N, ddot(md, N)));
        double lmp = dlen(mpar);
        d3 dpsi_a = dcross(pb, py), dpsi_b = dcross(py, pa);
        d3 dpsi_p = dscl(dadd(dadd(md, dpsi_a), dpsi_b), -1.0);
        double tt = (double)tu;
        d3 S = dadd(A, dscl(dsub(B, A), tt));
        double nsp = ddot(N, dsub(S, P));
        double lamd = ddot(N, dsub(d_of(cj), P)) / nsp;
        d3 dydt = dsub(dscl(dsub(B, A), lamd), dscl(dsub(S, P), lamd * ddot(N, dsub(B, A)) / nsp));
        double pe = (double)edge_weight(pre, E, Q, e) / (double)Q;
        double W = hw * (double)(vp - vm) * dlen(dydt) / (lmp * pe);
        dacc(g->d_pos_se, V, ed[0], dscl(dpsi_a, W));
        dacc(g->d_pos_se, V, ed[1], dscl(dpsi_b, W));
        double gb[3] = {0, 0, 0};
        chain_hit(&G, dscl(dpsi_p, W), gb, g->d_pos_se, V);
    }
}

/* Camera-silhouette term, primary edge sample m. */
static void primary_sample(const rctx *C, uint64_t seed, int64_t m, int64_t M, const double *dLdI,
                           gbuf *g, orc_counts *cnt) {
    const orc_scene *s = C->s;
    int V = s->V, E = C->E;
    if (C->pe_Q == 0) return;
    uint32_t wds[44];
    for (uint32_t b = 0; b < 11; ++b)
        orc_philox((uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)m, b, 2, 0, wds + 4 * b);
    uint64_t target = mulhi64(((uint64_t)wds[1] << 32) | wds[0], C->pe_Q);
    int32_t e = cdf_pick(C->pe_prefix, E, target);
    const int32_t *ed = C->edges + 4 * e;
    float tu = u01(wds[2]);
    f3 a = fpos(s, ed[0]), b = fpos(s, ed[1]);
    float ax, ay, bx, by;
    if (!project_f(s, a, &ax, &ay) || !project_f(s, b, &bx, &by)) return;
    float qx = ax + tu * (bx - ax), qy = ay + tu * (by - ay);
    float fpx = floorf(qx), fpy = floorf(qy);
    if (!(fpx >= 0.0f && fpx < (float)s->W && fpy >= 0.0f && fpy < (float)s->H)) return;
    f3 cam = {s->cam[0], s->cam[1], s->cam[2]};
    f3 mv = fcross(fsub(a, cam), fsub(b, cam));
    float gx = mv.x, gy = -mv.y;
    float gl = sqrtf(gx * gx + gy * gy);
    if (gl == 0.0f) return;
    float nx = gx / gl, ny = gy / gl;
    float lu[2 * MAXL];
    for (int j = 0; j < s->n_lights; ++j) { lu[2 * j] = u01(wds[4 + 2 * j]); lu[2 * j + 1] = u01(wds[5 + 2 * j]); }
    double f[2][3];
    for (int side = 0; side < 2; ++side) {
        float sg = side == 0 ? 1.0f : -1.0f;
        float px = qx + sg * (EDGE_OFF_PX * nx), py = qy + sg * (EDGE_OFF_PX * ny);
        sdec D;
        decide(C, px, py, lu, &D, cnt);
        sample_value(C, cam, camera_dir(s, px, py), &D, f[side]);
    }
    if (cnt) cnt->edge_primary += 2;
    int pix = (int)fpy * s->W + (int)fpx;
    const double *G = dLdI + 3 * (size_t)pix;
    double df = G[0] * (f[0][0] - f[1][0]) + G[1] * (f[0][1] - f[1][1]) + G[2] * (f[0][2] - f[1][2]);
    if (df == 0.0) return;
    /* value path in double */
    d3 A = dpos(s, ed[0]), B = dpos(s, ed[1]), Cd = d_of(cam);
    double ps = s->pix_scale;
    double qxd = (double)qx, qyd = (double)qy;
    d3 dq = dmk((qxd - 0.5 * s->W) * ps, (0.5 * s->H - qyd) * ps, -1.0);
    d3 md = dcross(dsub(A, Cd), dsub(B, Cd));
    double gradn = ps * sqrt(md.x * md.x + md.y * md.y);
    d3 ra = dsub(A, Cd), rb = dsub(B, Cd);
    double pax = 0.5 * s->W + (ra.x / -ra.z) / ps, pay = 0.5 * s->H - (ra.y / -ra.z) / ps;
    double pbx = 0.5 * s->W + (rb.x / -rb.z) / ps, pby = 0.5 * s->H - (rb.y / -rb.z) / ps;
    double len = sqrt((pbx - pax) * (pbx - pax) + (pby - pay) * (pby - pay));
    double pe = (double)edge_weight(C->pe_prefix, E, C->pe_Q, e) / (double)C->pe_Q;
    double W = df * len / (pe * gradn * (double)M);
    d3 dpsi_a = dcross(rb, dq), dpsi_b = dcross(dq, ra);
    dacc(g->d_pos_pe, V, ed[0], dscl(dpsi_a, W));
    dacc(g->d_pos_pe, V, ed[1], dscl(dpsi_b, W));
}

static void *job_run(void *arg) {
    job *J = arg;
    rctx *C = J->C;
    const orc_scene *s = C->s;
    int nl = s->n_lights;
    f3 cam = {s->cam[0], s->cam[1], s->cam[2]};
    if (J->mode == 5) {
        int64_t M = (int64_t)s->W * s->H;
        for (int64_t m = J->s0; m < J->s1; ++m) primary_sample(C, J->seed, m, M, J->dLdI, &J->g, &J->cnt);
        return NULL;
    }
    if (J->mode == 7) {      /* auxiliary buffers of selected pixels */
        for (int64_t i = J->s0; i < J->s1; ++i) {
            int pix = J->pix[i];
            int px = pix % s->W, py = pix / s->W;
            double acc[7] = {0, 0, 0, 0, 0, 0, 0};
            for (int k = 0; k < J->spp; ++k) {
                int64_t sidx = (int64_t)pix * J->spp + k;
                uint32_t w[44];
                camera_words(J->seed, (uint32_t)sidx, w);
                float qx = (float)px + u01(w[0]), qy = (float)py + u01(w[1]);
                f3 d = camera_dir(s, qx, qy);
                sample_aov(C, cam, d, acc);
            }
            for (int c = 0; c < 7; ++c) J->pix_out[7 * i + c] = acc[c] / J->spp;
        }
        return NULL;
    }
    if (J->mode == 6) {      /* selected pixels */
        for (int64_t i = J->s0; i < J->s1; ++i) {
            int pix = J->pix[i];
            int px = pix % s->W, py = pix / s->W;
            double acc[3] = {0, 0, 0};
            for (int k = 0; k < J->spp; ++k) {
                int64_t sidx = (int64_t)pix * J->spp + k;
                uint32_t w[44];
                camera_words(J->seed, (uint32_t)sidx, w);
                float lu[2 * MAXL];
                for (int j = 0; j < nl; ++j) { lu[2 * j] = u01(w[2 + 2 * j]); lu[2 * j + 1] = u01(w[3 + 2 * j]); }
                float qx = (float)px + u01(w[0]), qy = (float)py + u01(w[1]);
                sdec D;
                decide(C, qx, qy, lu, &D, &J->cnt);
                double c[3];
                sample_value(C, cam, camera_dir(s, qx, qy), &D, c);
                acc[0] += c[0]; acc[1] += c[1]; acc[2] += c[2];
            }
            for (int c = 0; c < 3; ++c) J->pix_out[3 * i + c] = acc[c] / J->spp;
        }
        return NULL;
    }
    for (int64_t sidx = J->s0; sidx < J->s1; ++sidx) {
        int64_t pix = sidx / J->spp;
        int px = (int)(pix % s->W), py = (int)(pix / s->W);
        uint32_t w[44];
        camera_words(J->seed, (uint32_t)sidx, w);
        float lu[2 * MAXL];
        for (int j = 0; j < nl; ++j) { lu[2 * j] = u01(w[2 + 2 * j]); lu[2 * j + 1] = u01(w[3 + 2 * j]); }
        float qx = (float)px + u01(w[0]), qy = (float)py + u01(w[1]);
        f3 d = camera_dir(s, qx, qy);
        sdec D;
        if (J->mode == 2 || J->mode == 4) rec_to_dec(C, J->rec_in + ORC_REC_WORDS * sidx, lu, &D);
        else decide(C, qx, qy, lu, &D, &J->cnt);
        if (J->mode == 1) {
            int32_t *r = J->rec_out + ORC_REC_WORDS * sidx;
            memset(r, 0, sizeof(int32_t) * ORC_REC_WORDS);
            r[0] = D.tri;
            if (D.tri >= 0) {
                r[1] = D.front | (D.spec_on << 1) | 4;
                r[2] = (int32_t)(uint32_t)D.vis;
                r[3] = (int32_t)(uint32_t)D.cs_on;
                r[4] = (int32_t)(uint32_t)D.cl_on;
                for (int j = 0; j < nl; ++j) r[5 + j / 16] |= (int32_t)((uint32_t)D.gsel[j] << (2 * (j % 16)));
                r[7] = D.tex_ix;
                r[8] = D.tex_iy;
            }
            continue;
        }
        if (J->mode == 0 || J->mode == 2) {
            double c[3];
            sample_value(C, cam, d, &D, c);
            for (int k = 0; k < 3; ++k) J->image[3 * pix + k] += c[k];
            continue;
        }
        /* backward */
        if (D.tri < 0) continue;
        double wgt[3];
        for (int k = 0; k < 3; ++k) wgt[k] = J->dLdI[3 * pix + k] / J->spp;
        if (J->mode == 4 || (J->flags & 1)) sample_adjoint(C, cam, d, &D, wgt, &J->g);
        if (J->mode == 3 && (J->flags & 4)) sample_secondary(C, J->seed, sidx, cam, d, &D, wgt, &J->g, &J->cnt);
    }
    return NULL;
}

/* run mode over [0, total) split into nthreads contiguous ranges; ranges are
 * cut on pixel boundaries (multiples of align) so forward writes never race. */
static void run_jobs(rctx *C, int mode, uint64_t seed, int32_t spp, int64_t total, int64_t align,
                     int nthreads, job *proto, job **jobs_out) {
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    job *jobs = calloc((size_t)nthreads, sizeof(job));
    pthread_t th[256];
    int64_t units = (total + align - 1) / align;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *proto;
        jobs[t].C = C; jobs[t].mode = mode; jobs[t].seed = seed; jobs[t].spp = spp;
        int64_t u0 = units * t / nthreads, u1 = units * (t + 1) / nthreads;
        jobs[t].s0 = u0 * align; jobs[t].s1 = u1 * align < total ? u1 * align : total;
        memset(&jobs[t].cnt, 0, sizeof(orc_counts));
        if (mode >= 3) gbuf_alloc(&jobs[t].g, C->s->V, C->s->n_lights, C->s->spec_res);
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, job_run, &jobs[t]);
    job_run(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    *jobs_out = jobs;
}

static void sum_counts(job *jobs, int n, orc_counts *out) {
    if (!out) return;
    memset(out, 0, sizeof(*out));
    for (int t = 0; t < n; ++t) {
        out->camera += jobs[t].cnt.camera; out->shadow += jobs[t].cnt.shadow;
        out->edge_primary += jobs[t].cnt.edge_primary; out->edge_secondary += jobs[t].cnt.edge_secondary;
    }
}

static int clamp_threads(int n) { return n < 1 ? 1 : (n > 256 ? 256 : n); }

int orc_render(const orc_scene *s, uint64_t seed, int32_t spp, int32_t nthreads,
               double *image, orc_counts *counts) {
    if (spp <= 0) return -1;
    rctx C;
    if (rctx_init(&C, s, 0)) return -1;
    nthreads = clamp_threads(nthreads);
    int64_t npix = (int64_t)s->W * s->H;
    memset(image, 0, sizeof(double) * 3 * (size_t)npix);
    job proto; memset(&proto, 0, sizeof(proto));
    proto.image = image;
    job *jobs;
    run_jobs(&C, 0, seed, spp, npix * spp, spp, nthreads, &proto, &jobs);
    for (int64_t i = 0; i < 3 * npix; ++i) image[i] /= spp;
    sum_counts(jobs, nthreads, counts);
    free(jobs);
    rctx_free(&C);
    return 0;
}

int orc_render_pixels(const orc_scene *s, uint64_t seed, int32_t spp,
                      int32_t n, const int32_t *pix, int32_t nthreads, double *out) {
    if (spp <= 0) return -1;
    rctx C;
    if (rctx_init(&C, s, 0)) return -1;
    nthreads = clamp_threads(nthreads);
    job proto; memset(&proto, 0, sizeof(proto));
    proto.pix = pix; proto.pix_out = out;
    job *jobs;
    run_jobs(&C, 6, seed, spp, n, 1, nthreads, &proto, &jobs);
    free(jobs);
    rctx_free(&C);
    return 0;
}

int orc_aov_pixels(const orc_scene *s, uint64_t seed, int32_t spp,
                   int32_t n, const int32_t *pix, int32_t nthreads, double *out) {
    if (spp <= 0) return -1;
    rctx C;
    if (rctx_init(&C, s, 0)) return -1;
    nthreads = clamp_threads(nthreads);
    job proto; memset(&proto, 0, sizeof(proto));
    proto.pix = pix; proto.pix_out = out;
    job *jobs;
    run_jobs(&C, 7, seed, spp, n, 1, nthreads, &proto, &jobs);
    free(jobs);
    rctx_free(&C);
    return 0;
}

int orc_record_decisions(const orc_scene *s, uint64_t seed, int32_t spp,
                         int32_t nthreads, int32_t *rec) {
    if (spp <= 0 || s->n_lights > 32) return -1;
    rctx C;
    if (rctx_init(&C, s, 0)) return -1;
    nthreads = clamp_threads(nthreads);
    job proto; memset(&proto, 0, sizeof(proto));
    proto.rec_out = rec;
    job *jobs;
    run_jobs(&C, 1, seed, spp, (int64_t)s->W * s->H * spp, spp, nthreads, &proto, &jobs);
    free(jobs);
    rctx_free(&C);
    return 0;
}

int orc_render_frozen(const orc_scene *s, uint64_t seed, int32_t spp,
                      const int32_t *rec, int32_t nthreads, double *image) {
    if (spp <= 0) return -1;
    rctx C;
    if (rctx_init(&C, s, 0)) return -1;
    nthreads = clamp_threads(nthreads);
    int64_t npix = (int64_t)s->W * s->H;
    memset(image, 0, sizeof(double) * 3 * (size_t)npix);
    job proto; memset(&proto, 0, sizeof(proto));
    proto.image = image; proto.rec_in = rec;
    job *jobs;
    run_jobs(&C, 2, seed, spp, npix * spp, spp, nthreads, &proto, &jobs);
    for (int64_t i = 0; i < 3 * npix; ++i) image[i] /= spp;
    free(jobs);
    rctx_free(&C);
    return 0;
}

/* d_nrm (vertex-normal adjoint) -> positions, through n_k = N_k/|N_k|,
 * N_k = sum_f N_f, N_f = (v1 - v0) x (v2 - v0). */
static void normal_chain(const rctx *C, const double *d_nrm, double *d_pos) {
    const orc_scene *s = C->s;
    int V = s->V;
    double *gN = calloc((size_t)3 * V, sizeof(double));
    for (int i = 0; i < V; ++i) {
        if (C->nrm_len[i] <= 0) continue;
        d3 n = dmk(C->nrm_d[i], C->nrm_d[V + i], C->nrm_d[2 * V + i]);
        d3 g = dmk(d_nrm[i], d_nrm[V + i], d_nrm[2 * V + i]);
        d3 r = dnorm_adj(g, n, C->nrm_len[i]);
        gN[i] = r.x; gN[V + i] = r.y; gN[2 * V + i] = r.z;
    }
    for (int f = 0; f < s->F; ++f) {
        const int32_t *t = s->faces + 3 * f;
        d3 g = dmk(0, 0, 0);
        for (int k = 0; k < 3; ++k) g = dadd(g, dmk(gN[t[k]], gN[V + t[k]], gN[2 * V + t[k]]));
        d3 v0 = dpos(s, t[0]);
        d3 a = dsub(dpos(s, t[1]), v0), b = dsub(dpos(s, t[2]), v0);
        d3 ga = dcross(b, g), gb = dcross(g, a);
        dacc(d_pos, V, t[1], ga);
        dacc(d_pos, V, t[2], gb);
        dacc(d_pos, V, t[0], dscl(dadd(ga, gb), -1.0));
    }
    free(gN);
}

static void reduce_grads(rctx *C, job *jobs, int n, orc_grads *g, int with_edges) {
    const orc_scene *s = C->s;
    int V = s->V, nl = s->n_lights, R = s->spec_res;
    double *d_nrm = calloc((size_t)3 * V, sizeof(double));
    double *d_int = calloc((size_t)3 * V, sizeof(double));
    double *d_pe = calloc((size_t)3 * V, sizeof(double));
    double *d_se = calloc((size_t)3 * V, sizeof(double));
    if (g->d_light) memset(g->d_light, 0, sizeof(double) * 3 * nl);
    if (g->d_spec) memset(g->d_spec, 0, sizeof(double) * R * R);
    if (g->d_alb) memset(g->d_alb, 0, sizeof(double) * 3 * V);
    for (int t = 0; t < n; ++t) {
        gbuf *b = &jobs[t].g;
        if (g->d_light) for (int i = 0; i < 3 * nl; ++i) g->d_light[i] += b->d_light[i];
        if (g->d_spec) for (int i = 0; i < R * R; ++i) g->d_spec[i] += b->d_spec[i];
        for (int i = 0; i < 3 * V; ++i) {
            if (g->d_alb) g->d_alb[i] += b->d_alb[i];
            d_nrm[i] += b->d_nrm[i];
            d_int[i] += b->d_pos[i];
            d_pe[i] += b->d_pos_pe[i];
            d_se[i] += b->d_pos_se[i];
        }
    }
    normal_chain(C, d_nrm, d_int);
    (void)with_edges;
    for (int i = 0; i < 3 * V; ++i) {
        if (g->d_pos) g->d_pos[i] = d_int[i] + d_pe[i] + d_se[i];
        if (g->d_pos_interior) g->d_pos_interior[i] = d_int[i];
        if (g->d_pos_primary) g->d_pos_primary[i] = d_pe[i];
        if (g->d_pos_secondary) g->d_pos_secondary[i] = d_se[i];
    }
    free(d_nrm); free(d_int); free(d_pe); free(d_se);
}

int orc_backward(const orc_scene *s, uint64_t seed, int32_t spp,
                 const double *dLdI, int32_t flags, int32_t nthreads,
                 orc_grads *g, orc_counts *counts) {
    if (spp <= 0) return -1;
    rctx C;
    if (rctx_init(&C, s, (flags & 6) != 0)) return -1;
    nthreads = clamp_threads(nthreads);
    int64_t npix = (int64_t)s->W * s->H;
    job proto; memset(&proto, 0, sizeof(proto));
    proto.dLdI = dLdI; proto.flags = flags;
    job *jobs;
    run_jobs(&C, 3, seed, spp, npix * spp, spp, nthreads, &proto, &jobs);
    orc_counts c1; sum_counts(jobs, nthreads, &c1);
    if (flags & 2) {
        job *pj;
        run_jobs(&C, 5, seed, spp, npix, 1, nthreads, &proto, &pj);
        /* fold primary-edge buffers into the first batch before reducing */
        for (int t = 0; t < nthreads; ++t) {
            for (int i = 0; i < 3 * s->V; ++i) jobs[t].g.d_pos_pe[i] += pj[t].g.d_pos_pe[i];
            c1.edge_primary += pj[t].cnt.edge_primary; c1.camera += pj[t].cnt.camera; c1.shadow += pj[t].cnt.shadow;
            gbuf_free(&pj[t].g);
        }
        free(pj);
    }
    if (counts) *counts = c1;
    reduce_grads(&C, jobs, nthreads, g, 1);
    for (int t = 0; t < nthreads; ++t) gbuf_free(&jobs[t].g);
    free(jobs);
    rctx_free(&C);
    return 0;
}

int orc_backward_frozen(const orc_scene *s, uint64_t seed, int32_t spp,
                        const int32_t *rec, const double *dLdI, int32_t nthreads,
                        orc_grads *g) {
    if (spp <= 0) return -1;
    rctx C;
    if (rctx_init(&C, s, 0)) return -1;
    nthreads = clamp_threads(nthreads);
    int64_t npix = (int64_t)s->W * s->H;
    job proto; memset(&proto, 0, sizeof(proto));
    proto.dLdI = dLdI; proto.rec_in = rec; proto.flags = 1;
    job *jobs;
    run_jobs(&C, 4, seed, spp, npix * spp, spp, nthreads, &proto, &jobs);
    reduce_grads(&C, jobs, nthreads, g, 0);
    for (int t = 0; t < nthreads; ++t) gbuf_free(&jobs[t].g);
    free(jobs);
    rctx_free(&C);
    return 0;
}
