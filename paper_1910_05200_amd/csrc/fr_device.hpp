// Device-side math for the light-stage renderer (gfx950, wave64).
//
// Two kinds of arithmetic live here:
//  * decisions: every comparison whose outcome is an integer (which triangle
//    a ray hits, whether a shadow ray is blocked, which side is seen, which
//    edge a sample picks) is taken in fp32 with the operation order written
//    below and no contraction (the library is built with -ffp-contract=off);
//  * values: shading and its adjoint, templated on the scalar type.  The
//    bulk runs in fp32; the edge samples, which sit on silhouettes by
//    construction and shade at grazing angles, run in fp64, which MI355X
//    issues at the fp32 (non-packed) rate.
// The estimator is the Monte-Carlo lighting estimator F of the paper's
// Optimization paragraph with the Cook-Torrance reflectance of its Face
// Modeling paragraph; see include/facert.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fr {

constexpr float kHitMargin = 1e-5f;      // accepted hit within tri box +- this
constexpr float kBoxPad = 2e-5f;         // BVH boxes are padded by this
constexpr float kShadowTmin = 1e-4f;
constexpr float kShadowTmax = 1.0f - 1e-4f;
constexpr float kEdgeOffPx = 1e-3f;      // silhouette sides, in pixels
constexpr float kEdgeOffM = 2e-5f;       // shadow-boundary sides, in metres
constexpr float kQScale = 1048576.0f;    // 2^20 edge-weight quantisation
constexpr double kBeckmannM = 0.35;
constexpr double kPi = 3.14159265358979323846;
constexpr float kSlabGrow = 1.0000004f;  // far-time growth of the slab test (see traversal)
constexpr int kMaxLights = 64;

template <class T> struct vec3 { T x, y, z; };
using v3 = vec3<float>;
using d3 = vec3<double>;
__device__ __forceinline__ v3 mk(float x, float y, float z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
__device__ __forceinline__ d3 dk(double x, double y, double z) { d3 r; r.x = x; r.y = y; r.z = z; return r; }
template <class T> __device__ __forceinline__ vec3<T> vk(T x, T y, T z) { vec3<T> r; r.x = x; r.y = y; r.z = z; return r; }
template <class T> __device__ __forceinline__ vec3<T> cvt(v3 a) { return vk<T>((T)a.x, (T)a.y, (T)a.z); }
template <class T> __device__ __forceinline__ vec3<T> operator-(vec3<T> a, vec3<T> b) { return vk<T>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class T> __device__ __forceinline__ vec3<T> operator+(vec3<T> a, vec3<T> b) { return vk<T>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class T> __device__ __forceinline__ vec3<T> operator*(vec3<T> a, T s) { return vk<T>(a.x * s, a.y * s, a.z * s); }
template <class T> __device__ __forceinline__ T dot(vec3<T> a, vec3<T> b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
template <class T> __device__ __forceinline__ vec3<T> cross(vec3<T> a, vec3<T> b) {
    return vk<T>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <class T> __device__ __forceinline__ T len(vec3<T> a) { return sqrt(dot(a, a)); }
// adjoint of n = v/|v|: dL/dv from dL/dn
template <class T> __device__ __forceinline__ vec3<T> norm_adj(vec3<T> g, vec3<T> n, T l) {
    return (g - n * dot(n, g)) * ((T)1 / l);
}

// ------------------------------------------------------------- Philox ----
// Philox4x32-10 (Salmon et al., SC'11).
struct u4 { uint32_t x, y, z, w; };
__device__ __forceinline__ u4 philox(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
    uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    u4 r; r.x = c0; r.y = c1; r.z = c2; r.w = c3;
    return r;
}
__device__ __forceinline__ float u01(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

// ------------------------------------------------------ scene on device --
using Node = uint4;
struct Scene {
    int V, F, W, H, nl, res, n_nodes, E;
    float cam_x, cam_y, cam_z, ps;
    const int *faces;          // [F][3]
    const float *pos;          // [3][V]
    const float *nrm;          // [3][V]
    const float *alb;          // [3][V]
    const float *uv;           // [2][V]
    const Node *nodes;         // [n_nodes]: binary16 box + link (see the traversal)
    const float4 *tris;        // [3 F] by triangle index: v0 v1 v2, the index
    const float *lgeom;        // [nl][12]
    const float *lrgb;         // [nl][3]
    const float *spec;         // [res^2]
    const int *edges;          // [E][4]
    // sampling tables (compacted positive-weight entries)
    const int *pe_edge; const uint64_t *pe_prefix; const int *pe_n; const uint64_t *pe_Q;
    const int *se_edge; const uint64_t *se_prefix; const int *se_n; const uint64_t *se_Q;  // [nl][E]
    const int *pe_guide, *se_guide;   // cut-point guides: [E + 1], [nl][E + 1]
    const float4 *edge_rec;           // [E][5]: endpoints, face normals and first vertices, face ids
    const float4 *edge_pl;            // [E][2]: each face's unit normal and offset (see edge_weights_body)
    float *geo_R;                     // largest |coordinate| of the posed vertices (a bound for edge_pl)
};

__device__ __forceinline__ v3 vpos_raw(const float *pos, int V, int i) {
    return mk(pos[i], pos[V + i], pos[2 * V + i]);
}
__device__ __forceinline__ v3 vpos(const Scene &S, int i) {
    return mk(S.pos[i], S.pos[S.V + i], S.pos[2 * S.V + i]);
}
__device__ __forceinline__ v3 face_normal(const Scene &S, int f) {
    const int *t = S.faces + 3 * f;
    v3 v0 = vpos(S, t[0]);
    return cross(vpos(S, t[1]) - v0, vpos(S, t[2]) - v0);
}

// -------------------------------------------------- ray / triangle -------
// Moller-Trumbore, two-sided, inclusive barycentric bounds, open t range;
// the hit point must lie in the triangle's box widened by kHitMargin.
__device__ __forceinline__ bool ray_tri(v3 o, v3 d, v3 v0, v3 v1, v3 v2, float tmin, float tmax,
                                        float &t_out, float &b1_out, float &b2_out, float &det_out) {
    v3 e1 = v1 - v0, e2 = v2 - v0;
    v3 pv = cross(d, e2);
    float det = dot(e1, pv);
    if (det == 0.0f) return false;
    float inv = 1.0f / det;
    v3 tv = o - v0;
    float b1 = dot(tv, pv) * inv;
    if (!(b1 >= 0.0f && b1 <= 1.0f)) return false;
    v3 qv = cross(tv, e1);
    float b2 = dot(d, qv) * inv;
    if (!(b2 >= 0.0f && b1 + b2 <= 1.0f)) return false;
    float t = dot(e2, qv) * inv;
    if (!(t > tmin && t < tmax)) return false;
    v3 P = mk(o.x + t * d.x, o.y + t * d.y, o.z + t * d.z);
    float lo, hi;
    lo = fminf(fminf(v0.x, v1.x), v2.x) - kHitMargin; hi = fmaxf(fmaxf(v0.x, v1.x), v2.x) + kHitMargin;
    if (!(P.x >= lo && P.x <= hi)) return false;
    lo = fminf(fminf(v0.y, v1.y), v2.y) - kHitMargin; hi = fmaxf(fmaxf(v0.y, v1.y), v2.y) + kHitMargin;
    if (!(P.y >= lo && P.y <= hi)) return false;
    lo = fminf(fminf(v0.z, v1.z), v2.z) - kHitMargin; hi = fmaxf(fmaxf(v0.z, v1.z), v2.z) + kHitMargin;
    if (!(P.z >= lo && P.z <= hi)) return false;
    t_out = t; b1_out = b1; b2_out = b2; det_out = det;
    return true;
}

// ---------------------------------------------------------- traversal ----
// The BVH is stored in depth-first order with escape links: after an
// internal node comes its left subtree; a miss (or a leaf) jumps to the
// escape index (a leaf's is the next node).  No stack is needed.
//
// A node is 16 bytes, one vector load: its box as six binary16 values,
// lo rounded toward -inf and hi toward +inf so that the stored box always
// contains the fp32 one (the triangle boxes padded by kBoxPad, internal
// boxes their unions), and a link word: >= 0 the escape index of an
// internal node, < 0 the complement of a leaf's triangle (its index in the
// mesh, which also indexes its record in tris, so a walk can skip its ray's
// own triangle before loading anything).  Boxes only
// cull, so a box test may err toward entering; it must never reject a box
// that holds an accepted hit.  (32-byte fp32 nodes save the six conversions
// but were slower: the walk is bound by the bytes each visit moves.)
//
// Why the slab test below cannot reject such a box: a ray/triangle test
// accepts only a hit point within the triangle's box widened by kHitMargin,
// and every box of the tree holds that triangle's box widened by kBoxPad =
// 2 kHitMargin, so the exact ray is at least kHitMargin (minus the hit
// point's own fp32 rounding, ~1e-7 m) inside every slab of every box on the
// way to an accepted hit.  In parameter units that is a margin of
// kHitMargin / |d_i| on each axis i.  The slab times are computed as
// fma(bound, 1/d_i, -o_i/d_i) with o_i/d_i rounded once per ray; their
// absolute error is below (|bound - o_i| + |o_i|) * 2^-22 / |d_i|, under
// 1e-6 / |d_i| for scenes within a few metres of the origin, an order of
// magnitude inside the margin.  The growth factor on the far time keeps the
// test conservative at the clamps (t = 0, t = thi) as well.
__device__ __forceinline__ float h2f(uint32_t bits16) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits16);
}
// binary16 bits of x rounded toward +inf (up) or -inf (down)
__device__ __forceinline__ uint32_t f2h_dir(float x, bool up) {
    _Float16 h = (_Float16)x;
    float b = (float)h;
    uint32_t u = __builtin_bit_cast(uint16_t, h);
    bool neg = (u & 0x8000u) != 0;
    if (up && b < x) u = neg ? u - 1u : u + 1u;              // b < x: x > 0 or |b| > |x|
    else if (!up && b > x) u = neg ? u + 1u : (u == 0u ? 0x8001u : u - 1u);
    return u;
}
struct NBox { float lx, ly, lz, hx, hy, hz; };
__device__ __forceinline__ NBox node_box(const Node &q) {
    NBox b;
    b.lx = h2f(q.x & 0xffffu); b.ly = h2f(q.x >> 16); b.lz = h2f(q.y & 0xffffu);
    b.hx = h2f(q.y >> 16); b.hy = h2f(q.z & 0xffffu); b.hz = h2f(q.z >> 16);
    return b;
}
__device__ __forceinline__ Node make_node(float lx, float ly, float lz, float hx, float hy, float hz, int link) {
    Node q;
    q.x = f2h_dir(lx, false) | (f2h_dir(ly, false) << 16);
    q.y = f2h_dir(lz, false) | (f2h_dir(hx, true) << 16);
    q.z = f2h_dir(hy, true) | (f2h_dir(hz, true) << 16);
    q.w = (uint32_t)link;
    return q;
}
__device__ __forceinline__ int node_link(const Node &q) { return (int)q.w; }
// node i of the array, addressed with a 32-bit byte offset from the base
__device__ __forceinline__ Node load_node(const Node *nodes, int i) {
    const char *base = reinterpret_cast<const char *>(nodes);
    return *reinterpret_cast<const Node *>(base + ((uint32_t)i << 4));
}

struct Ray {
    v3 o, d, id, oid;   // origin, direction, 1/direction (tiny components clamped), o/d
};
__device__ __forceinline__ float safe_inv(float x) {
    return 1.0f / (fabsf(x) < 1e-20f ? copysignf(1e-20f, x) : x);
}
__device__ __forceinline__ Ray make_ray(v3 o, v3 d) {
    Ray r; r.o = o; r.d = d; r.id = mk(safe_inv(d.x), safe_inv(d.y), safe_inv(d.z));
    r.oid = mk(o.x * r.id.x, o.y * r.id.y, o.z * r.id.z);
    return r;
}
__device__ __forceinline__ bool slab(const Ray &r, const NBox &b, float thi) {
    float tx0 = fmaf(b.lx, r.id.x, -r.oid.x), tx1 = fmaf(b.hx, r.id.x, -r.oid.x);
    float ty0 = fmaf(b.ly, r.id.y, -r.oid.y), ty1 = fmaf(b.hy, r.id.y, -r.oid.y);
    float tz0 = fmaf(b.lz, r.id.z, -r.oid.z), tz1 = fmaf(b.hz, r.id.z, -r.oid.z);
    float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), thi));
    return tn <= tf * kSlabGrow;
}

// The any-hit walk's slab test, the same decision as slab(r, node_box(q),
// 1) in fewer instructions.  With 1/d_i of either sign the rounded slab
// times keep the order of the bounds (fma with a fixed multiplier is
// monotone in the bound), so the smaller of an axis's two times is that of
// its near bound.  Each ray picks, per axis, its near and far bounds' 16-bit
// halves out of the node's words with one byte permutation (selectors set
// once per ray), which replaces the six minima and maxima.  The ray's own
// leaf enters as an empty box: its near time is raised to infinity through
// the clamp at t = 0 that the test makes anyway.
struct SlabSel { uint32_t x, y, z; };
__device__ __forceinline__ SlabSel slab_sel(const Ray &r) {
    // byte selectors of __builtin_amdgcn_perm(a, b, sel): 0-3 pick b's bytes, 4-7 a's
    SlabSel k;
    k.x = r.id.x >= 0.0f ? 0x03020504u : 0x05040302u;   // lx: q.x bytes 0-1, hx: q.y bytes 2-3
    k.y = r.id.y >= 0.0f ? 0x01000706u : 0x07060100u;   // ly: q.x bytes 2-3, hy: q.z bytes 0-1
    k.z = r.id.z >= 0.0f ? 0x03020504u : 0x05040302u;   // lz: q.y bytes 0-1, hz: q.z bytes 2-3
    return k;
}
__device__ __forceinline__ bool slab_any(const Ray &r, const SlabSel &k, const Node &q, float t0) {
    const uint32_t wx = __builtin_amdgcn_perm(q.x, q.y, k.x), wy = __builtin_amdgcn_perm(q.x, q.z, k.y),
                   wz = __builtin_amdgcn_perm(q.y, q.z, k.z);
    const float nx = fmaf(h2f(wx & 0xffffu), r.id.x, -r.oid.x), fx = fmaf(h2f(wx >> 16), r.id.x, -r.oid.x);
    const float ny = fmaf(h2f(wy & 0xffffu), r.id.y, -r.oid.y), fy = fmaf(h2f(wy >> 16), r.id.y, -r.oid.y);
    const float nz = fmaf(h2f(wz & 0xffffu), r.id.z, -r.oid.z), fz = fmaf(h2f(wz >> 16), r.id.z, -r.oid.z);
    const float tn = fmaxf(fmaxf(nx, ny), fmaxf(nz, t0));
    const float tf = fminf(fminf(fx, fy), fminf(fz, 1.0f));
    return tn <= tf * kSlabGrow;
}

struct Hit { int tri; float t, b1, b2, det; };
// work counters of one lane: box tests, triangle tests, shaded light samples
// Work counters of a lane: node tests, triangle tests, shaded samples, and
// node tests to take back (steps that a queued walk took past its ray's
// hit, see trace_any).
struct Work { uint32_t box = 0, tri = 0, shade = 0, box_back = 0; };

// closest hit, lexicographic (t, original triangle index)
__device__ inline Hit trace_closest(const Scene &S, v3 o, v3 d, Work &wk) {
    Ray r = make_ray(o, d);
    Hit h; h.tri = -1; h.t = INFINITY; h.b1 = h.b2 = h.det = 0.0f;
    int node = 0;
    while (node < S.n_nodes) {
        const Node q = load_node(S.nodes, node);
        int link = node_link(q);
        ++wk.box;
        if (slab(r, node_box(q), h.t)) {
            if (link < 0) {
                int leaf = ~link;
                float4 q0 = S.tris[3 * leaf], q1 = S.tris[3 * leaf + 1], q2 = S.tris[3 * leaf + 2];
                v3 v0 = mk(q0.x, q0.y, q0.z), v1 = mk(q0.w, q1.x, q1.y), v2 = mk(q1.z, q1.w, q2.x);
                int id = __float_as_int(q2.y);
                float t, b1, b2, det;
                ++wk.tri;
                if (ray_tri(o, d, v0, v1, v2, 0.0f, INFINITY, t, b1, b2, det)) {
                    if (t < h.t || (t == h.t && id < h.tri)) { h.tri = id; h.t = t; h.b1 = b1; h.b2 = b2; h.det = det; }
                }
            }
            node = node + 1;
        } else {
            node = link < 0 ? node + 1 : link;
        }
    }
    return h;
}

// any hit on o + t d, t in (kShadowTmin, kShadowTmax), ignoring triangle skip.
// The loop runs while any lane of the wave still walks (a wave-uniform exit),
// so the node tests can be counted per wave in a scalar register, from the
// mask of walking lanes, and added to one lane's counter at the end: a
// per-lane count costs a vector instruction on every step of a loop whose
// vector issue is its limit.  The total is the per-lane sum.
//
// Triangle tests are queued.  A lane whose ray enters a leaf's box (other
// than its own triangle's) appends the triangle, its own lane and the step
// to one list of the wave in LDS, and walks on.  Once the list holds
// kLeafRound entries, or no lane walks any more, the wave runs the listed
// tests in rounds, one entry per lane that entered whatever lane queued it, with
// the queuing lane's ray read from that lane's registers; a hit records its
// step in the queuing lane's LDS word with an atomic minimum.  Run where a
// lane met its leaf, a triangle test executed for the whole wave with about
// four of its lanes active and was more than half of the kernel's vector
// instructions; listed, a round fills the wave.  A lane whose triangle was
// hit stops; the steps it walked past that leaf decided nothing (any hit
// ends the ray), so the result is the walk's.  Triangle tests are counted
// as the walk makes them, those up to each ray's first hit; node tests past
// the hit are taken back from the hit's step.  A lane that had already left
// the tree before the round is charged as if it had walked on to it, so the
// node count is a lower bound of the walk's (0.2% low at paper scale).
// lq: the wave's 2 kLeafList + 64 LDS words (one 64-lane wave per block).
constexpr int kLeafList = 512;                // queued tests a wave's list holds
constexpr uint32_t kLeafRound = 48;           // listed tests that start the rounds
static_assert(kLeafRound + 64 <= kLeafList, "a step appends at most 64 entries");
__device__ inline bool trace_any(const Scene &S, v3 o, v3 d, int skip, Work &wk, uint32_t *__restrict__ lq) {
    uint32_t *const lstep = lq + kLeafList, *const lhit = lstep + kLeafList;
    const Ray r = make_ray(o, d);
    const int lane = (int)__lane_id();
    // the rounds deal the list to the lanes that entered (a lane whose
    // sample needs no ray, or past the queue's end, is not among them)
    const unsigned long long act = __ballot(true);
    const uint32_t n_act = (uint32_t)__popcll(act),
                   rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
    lhit[lane] = ~0u;                          // step of this lane's first hit
    int node = 0;
    bool hit = false;
    uint32_t boxes = 0, step = 0, cnt = 0;     // wave-uniform
    const int last = S.n_nodes - 1;
    int own = ~skip;                           // the ray's own leaf link
    asm volatile("" : "+v"(own));              // kept as is: one compare per step
    const SlabSel sel = slab_sel(r);
    for (;;) {
        for (;;) {                             // walk until the list is due
            const bool walk = node < S.n_nodes;
            const unsigned long long m = __ballot(walk);
            if (!m || cnt >= kLeafRound) break;
            boxes += (uint32_t)__popcll(m);
            // Every lane takes the step, with no branch around it: a lane
            // that has left the tree visits the last node, a leaf of the
            // depth-first layout, so its index only grows, and its test is
            // dropped.  (The branch cost a vector select and a mask copy
            // per step.)
            const Node q = load_node(S.nodes, min(node, last));
            const int link = node_link(q);
            const bool in = slab_any(r, sel, q, link == own ? INFINITY : 0.0f), leaf = link < 0;
            node = (in || leaf) ? node + 1 : link;
            const bool want = walk && in && leaf;
            // the mask of wanting lanes from one ballot per compare (leaf:
            // link < 0, predicate 40), ANDed in scalar registers; a ballot
            // of the combined flag is copied through a vector register
            const unsigned long long a = m & __builtin_amdgcn_ballot_w64(in) & __builtin_amdgcn_sicmp(link, 0, 40);
            if (want) {
                const uint32_t at = cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(a >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)a, 0u));
                lq[at] = ((uint32_t)~link << 6) | (uint32_t)lane;
                lstep[at] = step;
            }
            cnt += (uint32_t)__popcll(a);
            ++step;
        }
        if (!cnt) break;                       // no lane walks and nothing is listed
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (uint32_t base = 0; base < cnt; base += n_act) {
            const uint32_t g = base + rank;
            const bool has = g < cnt;
            const uint32_t e = has ? lq[g] : 0u;
            const int owner = (int)(e & 63u), t = (int)(e >> 6);
            const v3 oo = mk(__shfl(o.x, owner), __shfl(o.y, owner), __shfl(o.z, owner));
            const v3 dd = mk(__shfl(d.x, owner), __shfl(d.y, owner), __shfl(d.z, owner));
            if (has) {
                const float4 q0 = S.tris[3 * t], q1 = S.tris[3 * t + 1], q2 = S.tris[3 * t + 2];
                const v3 v0 = mk(q0.x, q0.y, q0.z), v1 = mk(q0.w, q1.x, q1.y), v2 = mk(q1.z, q1.w, q2.x);
                float tt, b1, b2, det;
                if (ray_tri(oo, dd, v0, v1, v2, kShadowTmin, kShadowTmax, tt, b1, b2, det))
                    atomicMin(&lhit[owner], lstep[g]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (uint32_t base = 0; base < cnt; base += n_act) {   // the tests the walk makes
            const uint32_t g = base + rank;
            if (g < cnt && lstep[g] <= lhit[lq[g] & 63u]) ++wk.tri;
        }
        const uint32_t hs = lhit[lane];
        if (hs != ~0u && !hit) {
            hit = true;
            node = S.n_nodes;                  // this lane's walk ends
            wk.box_back += step - hs - 1u;
        }
        cnt = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    // every lane that entered is active again: the first of them takes the wave's count
    if ((int)__lane_id() == __ffsll((unsigned long long)__builtin_amdgcn_read_exec()) - 1) wk.box += boxes;
    return hit;
}

// Closest hits of two rays from one origin in one traversal (the two sides
// of a camera-silhouette sample), each with its own nearest t as the slab
// bound; each result is that of trace_closest for the ray alone.
__device__ inline void trace_closest2(const Scene &S, v3 o, v3 d1, v3 d2, Hit &h1, Hit &h2, Work &wk) {
    const Ray r1 = make_ray(o, d1), r2 = make_ray(o, d2);
    h1.tri = -1; h1.t = INFINITY; h1.b1 = h1.b2 = h1.det = 0.0f;
    h2 = h1;
    int node = 0;
    while (node < S.n_nodes) {
        const Node q = load_node(S.nodes, node);
        const int link = node_link(q);
        const NBox b = node_box(q);
        const bool e1 = slab(r1, b, h1.t), e2 = slab(r2, b, h2.t);
        wk.box += 2;
        if (e1 || e2) {
            if (link < 0) {
                const int leaf = ~link;
                const float4 q0 = S.tris[3 * leaf], q1 = S.tris[3 * leaf + 1], q2 = S.tris[3 * leaf + 2];
                const v3 v0 = mk(q0.x, q0.y, q0.z), v1 = mk(q0.w, q1.x, q1.y), v2 = mk(q1.z, q1.w, q2.x);
                const int id = __float_as_int(q2.y);
                float t, b1, b2, det;
                if (e1) {
                    ++wk.tri;
                    if (ray_tri(r1.o, r1.d, v0, v1, v2, 0.0f, INFINITY, t, b1, b2, det) &&
                        (t < h1.t || (t == h1.t && id < h1.tri))) { h1.tri = id; h1.t = t; h1.b1 = b1; h1.b2 = b2; h1.det = det; }
                }
                if (e2) {
                    ++wk.tri;
                    if (ray_tri(r2.o, r2.d, v0, v1, v2, 0.0f, INFINITY, t, b1, b2, det) &&
                        (t < h2.t || (t == h2.t && id < h2.tri))) { h2.tri = id; h2.t = t; h2.b1 = b1; h2.b2 = b2; h2.det = det; }
                }
            }
            node = node + 1;
        } else {
            node = link < 0 ? node + 1 : link;
        }
    }
}

// Two rays from one origin in one traversal (the two sides of an edge
// sample: nearly the same direction).  Each node is loaded and decoded once
// and tested against each ray that is still open; the walk descends when
// either ray enters the node, and a ray tests a leaf's triangle only when
// its own box test passed.  A ray's box tests along the shared walk include
// those of its own walk, and its triangle tests those of its own walk, so
// each result is that of trace_any for the ray alone (the box tests are
// conservative: both equal the brute-force answer).
__device__ inline void trace_any2(const Scene &S, v3 o, v3 d1, v3 d2, int skip, bool &hit1, bool &hit2,
                                  Work &wk) {
    const Ray r1 = make_ray(o, d1), r2 = make_ray(o, d2);
    hit1 = hit2 = false;
    int node = 0;
    while (node < S.n_nodes && !(hit1 && hit2)) {
        const Node q = load_node(S.nodes, node);
        const int link = node_link(q);
        const NBox b = node_box(q);
        const bool e1 = !hit1 && slab(r1, b, 1.0f), e2 = !hit2 && slab(r2, b, 1.0f);
        wk.box += (hit1 ? 0u : 1u) + (hit2 ? 0u : 1u);
        if (e1 || e2) {
            if (link < 0) {
                const int leaf = ~link;
                const float4 q0 = S.tris[3 * leaf], q1 = S.tris[3 * leaf + 1], q2 = S.tris[3 * leaf + 2];
                if (__float_as_int(q2.y) != skip) {
                    const v3 v0 = mk(q0.x, q0.y, q0.z), v1 = mk(q0.w, q1.x, q1.y), v2 = mk(q1.z, q1.w, q2.x);
                    float t, b1, b2, det;
                    if (e1) { ++wk.tri; hit1 = ray_tri(r1.o, r1.d, v0, v1, v2, kShadowTmin, kShadowTmax, t, b1, b2, det); }
                    if (e2) { ++wk.tri; hit2 = ray_tri(r2.o, r2.d, v0, v1, v2, kShadowTmin, kShadowTmax, t, b1, b2, det); }
                }
            }
            node = node + 1;
        } else {
            node = link < 0 ? node + 1 : link;
        }
    }
}

// --------------------------------------------------- camera and lights ---
__device__ __forceinline__ v3 camera_dir(const Scene &S, float qx, float qy) {
    return mk((qx - 0.5f * (float)S.W) * S.ps, (0.5f * (float)S.H - qy) * S.ps, -1.0f);
}
struct Light { v3 c, e1, e2, n; float area; float r, g, b; };
__device__ __forceinline__ v3 light_point(const Light &L, float u, float v) {
    float a = u - 0.5f, b = v - 0.5f;
    return mk((L.c.x + a * L.e1.x) + b * L.e2.x, (L.c.y + a * L.e1.y) + b * L.e2.y,
              (L.c.z + a * L.e1.z) + b * L.e2.z);
}

// cdf_pick through a cut-point guide (guide[b] = cdf_pick(ceil(b Q / n)),
// b in [0, n]): the target's bucket floor(target n / Q) is estimated in
// fp64 (off by at most one), and the answer lies between the guide entries
// one bucket below and two above it, so the short search there returns
// cdf_pick's index exactly.
__device__ __forceinline__ int cdf_pick_guided(const uint64_t *prefix, const int *guide, int n, uint64_t Q,
                                               uint64_t target) {
    int b = (int)((double)target * (double)n / (double)Q);
    b = min(max(b, 0), n);
    int lo = guide[max(b - 1, 0)], hi = guide[min(b + 2, n)];
    while (lo < hi) {
        int mid = lo + (hi - lo + 1) / 2;
        if (prefix[mid] <= target) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// largest i < n with prefix[i] <= target (prefix[0] = 0, non-decreasing)
__device__ __forceinline__ int cdf_pick(const uint64_t *prefix, int n, uint64_t target) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = lo + (hi - lo + 1) / 2;
        if (prefix[mid] <= target) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// --------------------------------------------------- surface decisions ---
struct SurfDec {
    v3 p;          // shading point: origin of shadow rays
    v3 ng;         // e1 x e2 of the hit triangle (unflipped)
    v3 nu;         // interpolated vertex normal (unflipped, unnormalised)
    v3 wod;        // unit direction to the camera
    int tex_ix, tex_iy;  // bilinear texel cell of the specular map
    bool front;    // det > 0: the camera sees the side ng points to
    bool spec_on;  // viewer above the interpolated vertex normal
};

__device__ inline void surf_decide(const Scene &S, v3 o, const Hit &h, SurfDec &s) {
    const int *tr = S.faces + 3 * h.tri;
    int i0 = tr[0], i1 = tr[1], i2 = tr[2];
    v3 v0 = vpos(S, i0), v1 = vpos(S, i1), v2 = vpos(S, i2);
    float b1 = h.b1, b2 = h.b2;
    float b0 = (1.0f - b1) - b2;
    s.p = mk((b0 * v0.x + b1 * v1.x) + b2 * v2.x, (b0 * v0.y + b1 * v1.y) + b2 * v2.y,
             (b0 * v0.z + b1 * v1.z) + b2 * v2.z);
    const float *N = S.nrm; int V = S.V;
    v3 n0 = mk(N[i0], N[V + i0], N[2 * V + i0]);
    v3 n1 = mk(N[i1], N[V + i1], N[2 * V + i1]);
    v3 n2 = mk(N[i2], N[V + i2], N[2 * V + i2]);
    v3 nu = mk((b0 * n0.x + b1 * n1.x) + b2 * n2.x, (b0 * n0.y + b1 * n1.y) + b2 * n2.y,
               (b0 * n0.z + b1 * n1.z) + b2 * n2.z);
    float co = dot(nu, o - s.p);
    s.front = h.det > 0.0f;
    s.spec_on = s.front ? co > 0.0f : co < 0.0f;
    s.ng = cross(v1 - v0, v2 - v0);
    s.nu = nu;
    v3 c = o - s.p;
    float lc = sqrtf(dot(c, c));
    s.wod = mk(c.x / lc, c.y / lc, c.z / lc);
    // texel centres at (i + 1/2)/res
    float ux = (b0 * S.uv[i0] + b1 * S.uv[i1]) + b2 * S.uv[i2];
    float uy = (b0 * S.uv[V + i0] + b1 * S.uv[V + i1]) + b2 * S.uv[V + i2];
    s.tex_ix = (int)floorf((float)S.res * ux - 0.5f);
    s.tex_iy = (int)floorf((float)S.res * uy - 0.5f);
}

// Branches whose value is continuous but whose slope jumps: the clamps of
// cos_s and cos_l and the min of the V-cavity term.  Decided in fp32 from
// the sample's decision values so that every implementation differentiates
// the same branch.  The V-cavity comparisons G1, G2 >= 1 and G1 <= G2 are
// written with unnormalised dot products (positive factors cancel).
struct Branch { bool cs, cl; int gsel; };
__device__ __forceinline__ Branch light_branch(const SurfDec &sd, v3 ln, v3 y) {
    Branch b;
    v3 r = y - sd.p;
    v3 nn = sd.front ? sd.nu : mk(-sd.nu.x, -sd.nu.y, -sd.nu.z);
    b.cs = dot(nn, r) > 0.0f;
    b.cl = dot(ln, r) < 0.0f;
    b.gsel = 0;
    if (sd.spec_on && b.cs) {
        float lr = sqrtf(dot(r, r));
        v3 wi = mk(r.x / lr, r.y / lr, r.z / lr);
        v3 hs = wi + sd.wod;
        float a_s = dot(nn, wi), a_o = dot(nn, sd.wod);
        float nh = dot(nn, hs), oh2 = dot(sd.wod, hs), n2 = dot(sd.nu, sd.nu);
        float rhs = oh2 * n2;
        float g1 = (2.0f * nh) * a_o, g2 = (2.0f * nh) * a_s;
        if (g1 >= rhs && g2 >= rhs) b.gsel = 0;
        else if (a_o <= a_s) b.gsel = 1;
        else b.gsel = 2;
    }
    return b;
}

// light sample above the surface's tangent plane (two-sided)
__device__ __forceinline__ bool above(const SurfDec &s, v3 y) {
    float hz = dot(s.ng, y - s.p);
    return s.front ? hz > 0.0f : hz < 0.0f;
}

// ------------------------------------------------------- surface values --
template <class T> struct Surf {
    int i[3];
    T b[3];
    vec3<T> p;                 // shading point
    vec3<T> nu; T nlen;        // interpolated normal and its length
    vec3<T> ns;                // flipped, normalised shading normal
    vec3<T> wo; T olen; T cos_o;
    T A[3];
    T ks, tw[4], dks_du, dks_dv; int tex[4];
    vec3<T> N, dir, pv, e1xd; T det, ndotd, sg;   // barycentric chain
    bool spec_on;
};

template <class T>
__device__ inline void surf_value(const Scene &S, const float *spec_lds, v3 of, v3 df, const Hit &h,
                                  const SurfDec &dec, Surf<T> &s) {
    bool spec_on = dec.spec_on;
    const int *tr = S.faces + 3 * h.tri;
    int V = S.V;
    for (int k = 0; k < 3; ++k) s.i[k] = tr[k];
    v3 v0f = vpos(S, tr[0]), v1f = vpos(S, tr[1]), v2f = vpos(S, tr[2]);
    // barycentrics of the ray/plane solve in fp64 (grazing hits lose digits
    // as 1/det in fp32)
    d3 v0 = cvt<double>(v0f), v1 = cvt<double>(v1f), v2 = cvt<double>(v2f);
    d3 o = cvt<double>(of), d = cvt<double>(df);
    d3 e1 = v1 - v0, e2 = v2 - v0;
    d3 pvd = cross(d, e2);
    double det = dot(e1, pvd);
    d3 tv = o - v0;
    double inv = 1.0 / det;
    double b1 = dot(tv, pvd) * inv;
    d3 qv = cross(tv, e1);
    double b2 = dot(d, qv) * inv;
    double b0 = 1.0 - b1 - b2;
    s.b[0] = (T)b0; s.b[1] = (T)b1; s.b[2] = (T)b2;
    d3 pd = v0 * b0 + v1 * b1 + v2 * b2;
    s.p = vk<T>((T)pd.x, (T)pd.y, (T)pd.z);
    vec3<T> nu = vk<T>(0, 0, 0);
    for (int k = 0; k < 3; ++k)
        nu = nu + vk<T>((T)S.nrm[tr[k]], (T)S.nrm[V + tr[k]], (T)S.nrm[2 * V + tr[k]]) * s.b[k];
    s.nu = nu;
    s.nlen = len(nu);
    s.sg = h.det > 0.0f ? (T)1 : (T)-1;
    s.ns = nu * (s.sg / s.nlen);
    for (int c = 0; c < 3; ++c) {
        const float *a = S.alb + c * V;
        s.A[c] = s.b[0] * (T)a[tr[0]] + s.b[1] * (T)a[tr[1]] + s.b[2] * (T)a[tr[2]];
    }
    T ux = s.b[0] * (T)S.uv[tr[0]] + s.b[1] * (T)S.uv[tr[1]] + s.b[2] * (T)S.uv[tr[2]];
    T uy = s.b[0] * (T)S.uv[V + tr[0]] + s.b[1] * (T)S.uv[V + tr[1]] + s.b[2] * (T)S.uv[V + tr[2]];
    int R = S.res;
    // the cell is a decision (the slope jumps at texel centres)
    T x = (T)R * ux - (T)0.5, y = (T)R * uy - (T)0.5;
    int ix0 = dec.tex_ix, iy0 = dec.tex_iy;
    T fx = x - (T)ix0, fy = y - (T)iy0;
    int ixa = min(max(ix0, 0), R - 1), ixb = min(max(ix0 + 1, 0), R - 1);
    int iya = min(max(iy0, 0), R - 1), iyb = min(max(iy0 + 1, 0), R - 1);
    s.tex[0] = iya * R + ixa; s.tw[0] = ((T)1 - fx) * ((T)1 - fy);
    s.tex[1] = iya * R + ixb; s.tw[1] = fx * ((T)1 - fy);
    s.tex[2] = iyb * R + ixa; s.tw[2] = ((T)1 - fx) * fy;
    s.tex[3] = iyb * R + ixb; s.tw[3] = fx * fy;
    T T0 = spec_lds[s.tex[0]], T1 = spec_lds[s.tex[1]], T2 = spec_lds[s.tex[2]], T3 = spec_lds[s.tex[3]];
    s.ks = s.tw[0] * T0 + s.tw[1] * T1 + s.tw[2] * T2 + s.tw[3] * T3;
    s.dks_du = (T)R * (((T)1 - fy) * (T1 - T0) + fy * (T3 - T2));
    s.dks_dv = (T)R * (((T)1 - fx) * (T2 - T0) + fx * (T3 - T1));
    vec3<T> wv = cvt<T>(of) - s.p;
    s.olen = len(wv);
    s.wo = wv * ((T)1 / s.olen);
    s.cos_o = dot(s.ns, s.wo);
    vec3<T> e1t = cvt<T>(v1f - v0f), e2t = cvt<T>(v2f - v0f);
    s.N = cross(e1t, e2t);
    s.dir = cvt<T>(df);
    s.pv = cross(s.dir, e2t);
    s.e1xd = cross(e1t, s.dir);
    s.det = dot(e1t, s.pv);
    s.ndotd = dot(s.N, s.dir);
    s.spec_on = spec_on;
}

// Radiance of one visible light sample y and, if w is given, its
// reverse-mode adjoint.  c = l (A/pi cos_s + S) cos_l area/d^2,
// S = f_s cos_s = ks D G / (4 cos_o), Beckmann D, V-cavity G, F = 1.
template <class T> struct LAdj { vec3<T> gp, gns, gwo; T gA[3], gks, gl[3]; };

template <class T>
__device__ inline void shade_light(const Surf<T> &s, const Light &L, vec3<T> y, Branch br, const T *w, T out[3],
                                   LAdj<T> *adj) {
    const T one = 1, zero = 0, two = 2, four = 4, pi = (T)kPi;
    vec3<T> r = y - s.p;
    T d2 = dot(r, r), dist = sqrt(d2);
    vec3<T> wi = r * (one / dist);
    vec3<T> ln = cvt<T>(L.n);
    T area = (T)L.area;
    T cl_raw = -dot(ln, wi), cos_l = br.cl ? cl_raw : zero;
    T cs_raw = dot(s.ns, wi), cos_s = br.cs ? cs_raw : zero;
    T g = cos_l * area / d2;
    T D = 0, Fs = 0, ch = 0, oh = 0, lh = 1;   // Fs = S / ks
    int gsel = br.gsel;
    vec3<T> h = vk<T>(0, 0, 0);
    if (s.spec_on && br.cs) {
        vec3<T> hv = wi + s.wo;
        lh = len(hv);
        h = hv * (one / lh);
        ch = dot(s.ns, h);
        oh = dot(s.wo, h);
        T m2 = (T)(kBeckmannM * kBeckmannM), c2 = ch * ch;
        // Below the cut the exponent is under -790, where exp is exactly 0 in
        // fp32 and fp64 alike; testing first keeps 0/0 (c2^2 underflowing)
        // out of the grazing corner.  A NaN ch fails the test too.
        if (c2 * m2 > (T)1.25e-3) {
            D = exp(-(one - c2) / (c2 * m2)) / (pi * m2 * c2 * c2);
            // G/(4 cos_o) per branch of min(1, G1, G2), with cos_o cancelled
            // in the G1 branch: there the value cos_o can round to 0 at
            // grazing views while the fp32 decision still says "above".
            if (gsel == 0) Fs = D / (four * s.cos_o);
            else if (gsel == 1) Fs = D * ch / (two * oh);
            else Fs = D * ch * cos_s / (two * oh * s.cos_o);
        }
    }
    T Sv = s.ks * Fs;
    T lc[3] = {(T)L.r, (T)L.g, (T)L.b};
    for (int c = 0; c < 3; ++c) out[c] = lc[c] * (s.A[c] / pi * cos_s + Sv) * g;
    if (!adj) return;
    T Ld = 0, Lw = 0;
    for (int c = 0; c < 3; ++c) {
        adj->gl[c] = w[c] * (s.A[c] / pi * cos_s + Sv) * g;
        adj->gA[c] = w[c] * lc[c] * cos_s * g / pi;
        Ld += w[c] * lc[c] * s.A[c] / pi;
        Lw += w[c] * lc[c];
    }
    T g_cos_s = Ld * g;
    T g_S = Lw * g;
    T g_g = Ld * cos_s + Lw * Sv;
    adj->gks = g_S * Fs;
    T g_cos_l = g_g * area / d2;
    T g_d2 = -g_g * g / d2;
    vec3<T> g_wi = vk<T>(0, 0, 0), g_ns = vk<T>(0, 0, 0), g_wo = vk<T>(0, 0, 0);
    T g_cos_o = 0;
    if (D != zero) {   // where D is 0 every slope of S is 0 too
        T m2 = (T)(kBeckmannM * kBeckmannM);
        // dS/dD dD/dch = S (2/(m^2 ch^3) - 4/ch)
        T g_ch = g_S * Sv * (two / (m2 * ch * ch * ch) - four / ch);
        T g_oh = 0;
        if (gsel != 0) {   // S carries ch/oh in the G1 and G2 branches
            g_ch += g_S * Sv / ch;
            g_oh += -g_S * Sv / oh;
        }
        if (gsel != 1) g_cos_o += -g_S * Sv / s.cos_o;   // and 1/cos_o in the other two
        if (gsel == 2) g_cos_s += g_S * s.ks * D * ch / (two * oh * s.cos_o);
        g_ns = g_ns + h * g_ch;
        g_wo = g_wo + h * g_oh;
        vec3<T> g_h = s.ns * g_ch + s.wo * g_oh;
        vec3<T> g_hv = norm_adj(g_h, h, lh);
        g_wi = g_wi + g_hv;
        g_wo = g_wo + g_hv;
    }
    g_ns = g_ns + s.wo * g_cos_o;
    g_wo = g_wo + s.ns * g_cos_o;
    T g_cs = br.cs ? g_cos_s : zero;
    T g_cl = br.cl ? g_cos_l : zero;
    g_ns = g_ns + wi * g_cs;
    g_wi = g_wi + s.ns * g_cs;
    g_wi = g_wi - ln * g_cl;
    vec3<T> g_r = norm_adj(g_wi, wi, dist) + r * (two * g_d2);
    adj->gp = g_r * (T)-1;
    adj->gns = g_ns;
    adj->gwo = g_wo;
}

}  // namespace fr
