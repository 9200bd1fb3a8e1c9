/*
 * CPU oracle for the differentiable light-stage face renderer.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark load it; the product path never
 * does.  It shares no code with the GPU library.
 *
 * What it computes follows the paper (Dib et al., "Face Reflectance and
 * Geometry Modeling via Differentiable Ray Tracing"):
 *   - morphable geometry and albedo (Face Modeling paragraph: identity alpha,
 *     expression beta, albedo delta, pose [R t], vertex normals n_i);
 *   - the Monte-Carlo estimator F of the lighting equation (Optimization
 *     paragraph) with N = 20 oriented area lights, a Cook-Torrance BRDF
 *     (Lambertian albedo + gray specular texture) and shadow rays for
 *     self-shadows (Face Modeling, Optimization paragraphs);
 *   - the gradient of the photo-consistency loss E_data (Eq. 1) with respect
 *     to light colours, albedo, specular texels and vertex positions,
 *     including edge sampling of visibility discontinuities (Face Modeling
 *     paragraph, via the differentiable ray tracer it builds on).
 *
 * Precision: every continuous quantity is computed in IEEE double.  Every
 * floating-point comparison that decides an integer outcome (which triangle
 * a ray hits, whether a shadow ray is blocked, which side of a triangle is
 * seen, which edge a sample picks, which branch of a clamp or of the
 * V-cavity min a light sample takes, which texel cell it reads) is taken in
 * IEEE single precision with a fixed operation order and no contraction,
 * which is the precision the GPU kernels use.  Random numbers come from
 * Philox4x32-10 (Salmon et al. 2011).
 *
 * Parity pins (see the test suite): Philox known-answer vectors; blend
 * against a float64 matrix product; normals on flat and spherical grids;
 * intersection against exact rational arithmetic and brute force; Lambert's
 * polygon irradiance formula with and without a triangle shadow; a furnace
 * box; the textbook Beckmann lobe; central finite differences for the
 * interior gradient; for the edge terms, finite differences of exact
 * (quadrature, clipped-polygon Lambert) image and shadow integrals.
 */
#ifndef FACERT_ORACLE_H
#define FACERT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Scene for the estimator: geometry already posed. */
typedef struct {
    int32_t V, F;
    const int32_t *faces;     /* [F][3] vertex indices                          */
    const float   *pos;       /* [3][V] positions, single (decision inputs)     */
    const double  *pos_d;     /* [3][V] positions, double (value inputs)        */
    const double  *alb;       /* [3][V] per-vertex RGB albedo                   */
    const float   *uv;        /* [2][V] texture coordinates                     */
    int32_t W, H;
    float cam[3];             /* pinhole centre                                 */
    float pix_scale;          /* image-plane pixel size at unit depth           */
    int32_t n_lights;
    const float   *light_geom;/* [n][12] centre, e1, e2, unit emitting normal   */
    const double  *light_rgb; /* [n][3]                                         */
    int32_t spec_res;
    const double  *spec;      /* [res*res] row-major gray specular texels       */
} orc_scene;

typedef struct {
    double *d_light;          /* [n][3]                                   */
    double *d_spec;           /* [res*res]                                */
    double *d_pos;            /* [3][V] total dL/d(position)              */
    double *d_alb;            /* [3][V] dL/d(per-vertex albedo)           */
    double *d_pos_interior;   /* [3][V] optional: interior part (incl. normal chain) */
    double *d_pos_primary;    /* [3][V] optional: camera-silhouette edge part */
    double *d_pos_secondary;  /* [3][V] optional: shadow-boundary edge part  */
} orc_grads;

/* counts of rays traced by the last call on this thread */
typedef struct {
    int64_t camera, shadow, edge_primary, edge_secondary;
} orc_counts;

/* Philox4x32-10 block: key (k0,k1), counter (c0..c3) -> out[4]. */
void orc_philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                uint32_t c2, uint32_t c3, uint32_t out[4]);

/* R = Rz(rz) Ry(ry) Rx(rx) in double; row-major R[3*i+j]. */
void orc_rotation(const float pose[6], double R[9]);

/* v_model = mean + sum_k B_id[k] alpha_k + sum_k B_exp[k] beta_k (double,
 * k ascending, identity before expression); v = R v_model + t (double).
 * All arrays [3][V] (bases [K][3][V]).  v_model may be NULL. */
void orc_blend_geometry(int32_t V, int32_t n_id, int32_t n_exp,
                        const float *mean, const float *b_id, const float *b_exp,
                        const float *alpha, const float *beta, const float pose[6],
                        double *v_model, double *v);
void orc_blend_albedo(int32_t V, int32_t n_alb, const float *alb_mean,
                      const float *b_alb, const float *delta, double *A);

/* Vertex normals: normalize(sum over incident faces, ascending face index,
 * of (v1-v0) x (v2-v0)), in double from the given positions. */
void orc_vertex_normals(int32_t V, int32_t F, const int32_t *faces,
                        const double *pos, double *nrm);

/* Edge table: unique undirected edges sorted by (a, b) with a < b; each row
 * (a, b, f1, f2), f1 < f2 the adjacent faces, f2 = -1 on the boundary.
 * out must hold 3F rows.  Returns E, or -1 if an edge has > 2 faces. */
int32_t orc_build_edges(int32_t V, int32_t F, const int32_t *faces, int32_t *out);

/* Single-precision ray/triangle test (decision path).  Returns 1 on hit. */
int orc_ray_tri(const float o[3], const float d[3], const float v0[3],
                const float v1[3], const float v2[3], float tmin, float tmax,
                float *t, float *b1, float *b2, float *det);

/* Closest hit over all triangles (brute force, or through the oracle's own
 * BVH when use_bvh); returns the triangle index or -1.  t/b1/b2/det out. */
int32_t orc_closest_hit(const orc_scene *s, int use_bvh, const float o[3],
                        const float d[3], float *t, float *b1, float *b2, float *det);
/* Any hit on the segment o + t d, t in (1e-4, 1 - 1e-4), skipping 'skip'. */
int orc_any_hit(const orc_scene *s, int use_bvh, const float o[3],
                const float d[3], int32_t skip);

/* Forward render: image [H][W][3] in double.  Returns 0 or <0 on error. */
int orc_render(const orc_scene *s, uint64_t seed, int32_t spp, int32_t nthreads,
               double *image, orc_counts *counts);

/* Render a subset of pixels (list of pixel indices py*W+px); out [n][3]. */
int orc_render_pixels(const orc_scene *s, uint64_t seed, int32_t spp,
                      int32_t n, const int32_t *pix, int32_t nthreads, double *out);

/* Auxiliary buffers of n selected pixels (flat indices pix[i] = y*W + x):
 * out[i][7] = mean over the pixel's spp camera samples (the estimator's own
 * jitter and closest hits) of the first hit's albedo (RGB), unit shading
 * normal turned toward the camera (xyz) and distance from the camera;
 * misses contribute zeros.  These are the inputs of a denoiser, not part of
 * the estimator F. */
int orc_aov_pixels(const orc_scene *s, uint64_t seed, int32_t spp,
                   int32_t n, const int32_t *pix, int32_t nthreads, double *out);

/* Decision record of every camera sample (for frozen-decision checks), 9
 * int32 words: tri, flags (bit0 front-facing, bit1 specular lobe active,
 * bit2 hit), visibility mask, cos_s-clamp mask, cos_l-clamp mask, V-cavity
 * branches (2 bits per light, lights 0-15 then 16-31), texel cell x, y.
 * At most 32 lights. */
int orc_record_decisions(const orc_scene *s, uint64_t seed, int32_t spp,
                         int32_t nthreads, int32_t *rec);
/* Re-evaluate the estimator with decisions frozen from rec (value path only,
 * using s->pos_d, s->alb, s->light_rgb, s->spec as given). */
int orc_render_frozen(const orc_scene *s, uint64_t seed, int32_t spp,
                      const int32_t *rec, int32_t nthreads, double *image);

/* Adjoint of the loss whose image gradient is dLdI [H][W][3].  flags:
 * bit0 interior, bit1 camera-silhouette edges, bit2 shadow-boundary edges. */
int orc_backward(const orc_scene *s, uint64_t seed, int32_t spp,
                 const double *dLdI, int32_t flags, int32_t nthreads,
                 orc_grads *g, orc_counts *counts);
/* Interior adjoint with decisions frozen from rec (pins the adjoint against
 * finite differences of orc_render_frozen). */
int orc_backward_frozen(const orc_scene *s, uint64_t seed, int32_t spp,
                        const int32_t *rec, const double *dLdI, int32_t nthreads,
                        orc_grads *g);

#ifdef __cplusplus
}
#endif
#endif
