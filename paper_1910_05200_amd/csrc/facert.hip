// facert: differentiable light-stage face renderer for MI355X (gfx950).
//
// Kernels and the C-ABI declared in include/facert.h.  Build with
//   hipcc --offload-arch=gfx950 -O3 -ffp-contract=off -fPIC -shared
// (no contraction: the fp32 decision arithmetic must round every operation
// on its own, see fr_device.hpp).
//
// Per evaluation (fr_render):
//   k_blend, k_pose  morphable model and pose (Face Modeling paragraph),
//                    fp64 sums
//   k_normals        vertex normals, fixed-order gather over incident faces
//   k_refit_sub, k_refit_top  BVH boxes bottom-up (tree shape fixed at
//                    creation)
//   k_edge_weights   camera-silhouette and per-light shadow-candidate edges
//   k_edge_scan      integer CDFs of the edge weights (one block per table)
//   k_cam_init, k_cam_raster, k_cam_resolve, k_sh_propose, k_sh_trace, k_fwd_shade
//                    Monte-Carlo estimator F (Optimization paragraph): hit
//                    records, compacted shadow rays, Cook-Torrance shading
//   k_pixel_mean     fixed-order mean of each pixel's samples
// Adjoint (fr_backward), chunk by chunk over the camera samples:
//   k_render_adj     reverse mode of each camera sample's shading, scattered
//                    to lights/texels/albedo/normals/vertices
//   k_edge_secondary, k_edge_secondary_value
//                    shadow-boundary edge samples
//   k_edge_primary_{setup,vis,shade,scatter}
//                    camera-silhouette edge samples
//   k_normal_adj, k_chain_gather, k_param_partial, k_param_final
//                    normal chain, transposed blend and pose reductions
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/facert.h"
#include "fr_device.hpp"

using namespace fr;

// ====================================================================== //
//                               kernels                                  //
// ====================================================================== //

// ---------------------------------------------------------- blend -------
// v_model = mean + sum_k B_id[k] alpha_k + sum_k B_exp[k] beta_k  (fp64,
// k ascending, identity first); A = alb_mean + sum_k B_alb[k] delta_k
// (fp64).  One thread per (row, vertex), rows x, y, z of the geometry and
// r, g, b of the albedo on the grid's y axis, so that the 20k-vertex model
// spreads over ~1900 blocks; each k step reads one contiguous basis row,
// coalesced across the wave.  The geometry rows keep their fp64 sums for
// k_pose: v = R v_model + t (fp64).  Everything is rounded to fp32 once.
struct PoseArgs { double R[9]; double t[3]; };

// Every kernel's work is a body over one block-sized tile (bx, by): the
// __global__ wrappers below run one instance with the tile taken from the
// grid, the multi-instance launcher (k_multi) runs the tiles of many.
__device__ __forceinline__ void blend_body(int V, int n_id, int n_exp, int n_alb,
        const float *__restrict__ mean, const float *__restrict__ b_id, const float *__restrict__ b_exp,
        const float *__restrict__ alb_mean, const float *__restrict__ b_alb,
        const float *__restrict__ alpha, const float *__restrict__ beta, const float *__restrict__ delta,
        double *__restrict__ vm_d, float *__restrict__ vmodel, float *__restrict__ alb, int bx, int row,
        float *geo_R) {
    int i = bx * blockDim.x + threadIdx.x;
    if (bx == 0 && row == 0 && threadIdx.x == 0) *geo_R = 0.0f;   // pose_body takes the maximum
    if (i >= V) return;
    size_t V3 = (size_t)3 * V;
    if (row < 3) {
        size_t e = (size_t)row * V + i;
        double acc = (double)mean[e];
#pragma unroll 8
        for (int k = 0; k < n_id; ++k) acc = acc + (double)b_id[k * V3 + e] * (double)alpha[k];
#pragma unroll 8
        for (int k = 0; k < n_exp; ++k) acc = acc + (double)b_exp[k * V3 + e] * (double)beta[k];
        vm_d[e] = acc;
        vmodel[e] = (float)acc;
    } else {
        size_t e = (size_t)(row - 3) * V + i;
        double acc = (double)alb_mean[e];
#pragma unroll 8
        for (int k = 0; k < n_alb; ++k) acc = acc + (double)b_alb[k * V3 + e] * (double)delta[k];
        alb[e] = (float)acc;
    }
}
__global__ __launch_bounds__(64) void k_blend(int V, int n_id, int n_exp, int n_alb,
        const float *__restrict__ mean, const float *__restrict__ b_id, const float *__restrict__ b_exp,
        const float *__restrict__ alb_mean, const float *__restrict__ b_alb,
        const float *__restrict__ alpha, const float *__restrict__ beta, const float *__restrict__ delta,
        double *__restrict__ vm_d, float *__restrict__ vmodel, float *__restrict__ alb, float *geo_R) {
    blend_body(V, n_id, n_exp, n_alb, mean, b_id, b_exp, alb_mean, b_alb, alpha, beta, delta, vm_d, vmodel, alb,
               blockIdx.x, blockIdx.y, geo_R);
}

// Also the largest |coordinate| of the posed vertices, into *geo_R (zeroed
// by blend_body; one atomic maximum per wave on the bit pattern, which
// orders non-negative floats): the shadow-boundary proposals' plane
// pre-test scales its rounding bound by it.
__device__ __forceinline__ void pose_body(int V, const double *__restrict__ vm_d, const PoseArgs &P,
                                          float *__restrict__ pos, int bx, float *geo_R) {
    int i = bx * blockDim.x + threadIdx.x;
    float r = 0.0f;
    if (i < V) {
        double m[3] = {vm_d[i], vm_d[V + i], vm_d[2 * (size_t)V + i]};
        for (int c = 0; c < 3; ++c) {
            double v = ((P.R[3 * c] * m[0] + P.R[3 * c + 1] * m[1]) + P.R[3 * c + 2] * m[2]) + P.t[c];
            pos[(size_t)c * V + i] = (float)v;
            r = fmaxf(r, fabsf((float)v));
        }
    }
    for (int off = 32; off > 0; off >>= 1) r = fmaxf(r, __shfl_xor(r, off));
    if ((threadIdx.x & 63) == 0 && r > 0.0f) atomicMax((unsigned int *)geo_R, __float_as_uint(r));
}
__global__ __launch_bounds__(256) void k_pose(int V, const double *__restrict__ vm_d, PoseArgs P,
                                              float *__restrict__ pos, float *geo_R) {
    pose_body(V, vm_d, P, pos, blockIdx.x, geo_R);
}

// ---------------------------------------------------------- normals -----
// n_k = normalize(sum over incident faces, ascending index, of
// (v1 - v0) x (v2 - v0)), fp64 from the fp32 positions, rounded to fp32.
__device__ __forceinline__ void normals_body(int V, const int *__restrict__ faces,
        const int *__restrict__ vf_off, const int *__restrict__ vf_idx,
        const float *__restrict__ pos, float *__restrict__ nrm, float *__restrict__ nlen, int bx) {
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= V) return;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int q = vf_off[i]; q < vf_off[i + 1]; ++q) {
        const int *t = faces + 3 * vf_idx[q];
        double x0 = pos[t[0]], y0 = pos[V + t[0]], z0 = pos[2 * V + t[0]];
        double ax = (double)pos[t[1]] - x0, ay = (double)pos[V + t[1]] - y0, az = (double)pos[2 * V + t[1]] - z0;
        double bx = (double)pos[t[2]] - x0, by = (double)pos[V + t[2]] - y0, bz = (double)pos[2 * V + t[2]] - z0;
        sx = sx + (ay * bz - az * by);
        sy = sy + (az * bx - ax * bz);
        sz = sz + (ax * by - ay * bx);
    }
    double l = sqrt((sx * sx + sy * sy) + sz * sz);
    if (l > 0.0) { sx = sx / l; sy = sy / l; sz = sz / l; }
    nrm[i] = (float)sx; nrm[V + i] = (float)sy; nrm[2 * V + i] = (float)sz;
    nlen[i] = (float)l;
}
__global__ __launch_bounds__(256) void k_normals(int V, const int *__restrict__ faces,
        const int *__restrict__ vf_off, const int *__restrict__ vf_idx,
        const float *__restrict__ pos, float *__restrict__ nrm, float *__restrict__ nlen) {
    normals_body(V, faces, vf_off, vf_idx, pos, nrm, nlen, blockIdx.x);
}

// ------------------------------------------------------------ refit -----
// The tree's shape is fixed at creation; every evaluation recomputes its
// boxes.  The tree is cut into subtrees of at most kRefitLeaves leaves (a
// node range and a slot range each, depth-first layout) and the few nodes
// above them.  k_refit_sub: one block per subtree writes the triangle
// records and leaf boxes of its slots, then the internal boxes one height
// at a time with a block barrier between heights.  k_refit_top: one block,
// the top nodes by height.  No atomics and no device-wide fences.
constexpr int kRefitLeaves = 512;
struct SubTree { int node, slot, count, height; };

__device__ __forceinline__ void refit_union(Node *nodes, int n, int r, int esc) {
    NBox L = node_box(nodes[n + 1]), R = node_box(nodes[r]);
    nodes[n] = make_node(fminf(L.lx, R.lx), fminf(L.ly, R.ly), fminf(L.lz, R.lz),
                     fmaxf(L.hx, R.hx), fmaxf(L.hy, R.hy), fmaxf(L.hz, R.hz), esc);
}

__global__ __launch_bounds__(256) void k_refit_sub(const SubTree *__restrict__ subs, const int *__restrict__ faces,
        const float *__restrict__ pos, int V, const int *__restrict__ sorted_tri, const int *__restrict__ leaf_node,
        const int *__restrict__ height, const int *__restrict__ right, const int *__restrict__ escape,
        Node *nodes, float4 *__restrict__ tris) {
    const SubTree st = subs[blockIdx.x];
    for (int i = st.slot + threadIdx.x; i < st.slot + st.count; i += blockDim.x) {
        int f = sorted_tri[i];
        const int *t = faces + 3 * f;
        v3 a = vpos_raw(pos, V, t[0]), b = vpos_raw(pos, V, t[1]), c = vpos_raw(pos, V, t[2]);
        tris[3 * f] = make_float4(a.x, a.y, a.z, b.x);
        tris[3 * f + 1] = make_float4(b.y, b.z, c.x, c.y);
        tris[3 * f + 2] = make_float4(c.z, __int_as_float(f), 0.0f, 0.0f);
        nodes[leaf_node[i]] = make_node(fminf(fminf(a.x, b.x), c.x) - kBoxPad, fminf(fminf(a.y, b.y), c.y) - kBoxPad,
                                    fminf(fminf(a.z, b.z), c.z) - kBoxPad, fmaxf(fmaxf(a.x, b.x), c.x) + kBoxPad,
                                    fmaxf(fmaxf(a.y, b.y), c.y) + kBoxPad, fmaxf(fmaxf(a.z, b.z), c.z) + kBoxPad, ~f);
    }
    const int n_end = st.node + 2 * st.count - 1;
    for (int h = 1; h <= st.height; ++h) {
        __syncthreads();
        for (int n = st.node + threadIdx.x; n < n_end; n += blockDim.x)
            if (height[n] == h) refit_union(nodes, n, right[n], escape[n]);
    }
}

__global__ __launch_bounds__(256) void k_refit_top(int n_top, const int *__restrict__ top, const int *__restrict__ top_off,
        int top_levels, const int *__restrict__ right, const int *__restrict__ escape, Node *nodes) {
    for (int lv = 0; lv < top_levels; ++lv) {
        for (int k = top_off[lv] + threadIdx.x; k < top_off[lv + 1]; k += blockDim.x) {
            int n = top[k];
            refit_union(nodes, n, right[n], escape[n]);
        }
        __syncthreads();
    }
}

#include "fr_lbvh.hpp"

// ------------------------------------------------------- edge tables ----
__device__ __forceinline__ bool project(const Scene &S, v3 x, float &sx, float &sy) {
    v3 r = x - mk(S.cam_x, S.cam_y, S.cam_z);
    if (!(r.z < 0.0f)) return false;
    float nz = -r.z;
    sx = 0.5f * (float)S.W + (r.x / nz) / S.ps;
    sy = 0.5f * (float)S.H - (r.y / nz) / S.ps;
    return true;
}

// weights: table 0 = camera silhouettes (screen length), table 1+j = shadow
// candidates of light j (3D length).
// Besides the 80-byte record, each edge gets a 32-byte plane record for the
// proposals' pre-test: each face's unit normal u = N / |N| (N its fp32
// cross product, the one the exact silhouette test uses) and offset
// d = u . o (o its first vertex), NaN for a boundary edge's first face.
// For a shading point p, t = u . p - d approximates N . (p - o) / |N| within
// about 17 eps (|p|_inf + R) + eps |t| (R: largest |coordinate| of the
// posed mesh, eps = 2^-24), and the exact fp32 value of N . (p - o), as the
// silhouette test computes it, lies within 7 eps (|p|_inf + R) |N| of the
// real one.  So |t| > 64 eps (|p|_inf + R) + 4 eps |t| fixes the exact
// test's sign; when both faces' signs are fixed and equal, the exact test
// would reject the edge, and the proposal rejects it without the full
// record (a NaN, from a degenerate face or a boundary edge, fixes nothing).
__device__ __forceinline__ void edge_weights_body(const Scene &S, const float *__restrict__ lgeom,
        float *__restrict__ w, float4 *__restrict__ rec, float4 *__restrict__ pl, int tb) {
    const int e = tb * blockDim.x + threadIdx.x;
    if (e >= S.E) return;
    const int *ed = S.edges + 4 * e;
    v3 a = vpos(S, ed[0]), b = vpos(S, ed[1]);
    bool interior = ed[3] >= 0;
    v3 n1 = mk(0, 0, 0), n2 = mk(0, 0, 0), o1 = mk(0, 0, 0), o2 = mk(0, 0, 0);
    if (interior) {
        n1 = face_normal(S, ed[2]); n2 = face_normal(S, ed[3]);
        o1 = vpos(S, S.faces[3 * ed[2]]); o2 = vpos(S, S.faces[3 * ed[3]]);
    }
    // the edge's geometry for the shadow-boundary proposals, in one record
    rec[5 * e] = make_float4(a.x, a.y, a.z, b.x);
    rec[5 * e + 1] = make_float4(b.y, b.z, n1.x, n1.y);
    rec[5 * e + 2] = make_float4(n1.z, o1.x, o1.y, o1.z);
    rec[5 * e + 3] = make_float4(n2.x, n2.y, n2.z, o2.x);
    rec[5 * e + 4] = make_float4(o2.y, o2.z, __int_as_float(ed[2]), __int_as_float(ed[3]));
    if (interior) {
        const float l1 = sqrtf(dot(n1, n1)), l2 = sqrtf(dot(n2, n2));
        const v3 u1 = mk(n1.x / l1, n1.y / l1, n1.z / l1), u2 = mk(n2.x / l2, n2.y / l2, n2.z / l2);
        pl[2 * e] = make_float4(u1.x, u1.y, u1.z, dot(u1, o1));
        pl[2 * e + 1] = make_float4(u2.x, u2.y, u2.z, dot(u2, o2));
    } else {
        pl[2 * e] = make_float4(NAN, NAN, NAN, NAN);
        pl[2 * e + 1] = make_float4(NAN, NAN, NAN, NAN);
    }
    size_t E = (size_t)S.E;
    v3 cam = mk(S.cam_x, S.cam_y, S.cam_z);
    bool sil = true;
    if (interior) {
        float s1 = dot(n1, cam - o1), s2 = dot(n2, cam - o2);
        sil = (s1 > 0.0f) != (s2 > 0.0f);
    }
    float we = 0.0f, ax, ay, bx, by;
    if (sil && project(S, a, ax, ay) && project(S, b, bx, by)) {
        float dx = bx - ax, dy = by - ay;
        we = sqrtf(dx * dx + dy * dy);
    }
    w[e] = we;
    v3 ab = b - a;
    float l3 = sqrtf(dot(ab, ab));
    for (int j = 0; j < S.nl; ++j) {
        const float *g = lgeom + 12 * j;
        v3 c = mk(g[0], g[1], g[2]), e1 = mk(g[3], g[4], g[5]), e2 = mk(g[6], g[7], g[8]);
        bool cand = true;
        if (interior) {
            int posc = 0, negc = 0;
            for (int k = 0; k < 4; ++k) {
                float s1 = (k & 1) ? 0.5f : -0.5f, s2 = (k & 2) ? 0.5f : -0.5f;
                v3 x = mk((c.x + s1 * e1.x) + s2 * e2.x, (c.y + s1 * e1.y) + s2 * e2.y, (c.z + s1 * e1.z) + s2 * e2.z);
                int g1 = dot(n1, x - o1) > 0.0f, g2 = dot(n2, x - o2) > 0.0f;
                posc += g1 + g2; negc += 2 - g1 - g2;
            }
            cand = posc > 0 && negc > 0;
        }
        w[(size_t)(1 + j) * E + e] = cand ? l3 : 0.0f;
    }
}
__global__ __launch_bounds__(256) void k_edge_weights(Scene S, const float *__restrict__ lgeom,
        float *__restrict__ w, float4 *__restrict__ rec, float4 *__restrict__ pl) {
    edge_weights_body(S, lgeom, w, rec, pl, blockIdx.x);
}

// One block per table: the table's max weight wmax (block reduction), then
// q = 1 + floor(w / wmax * 2^20) for w > 0, exclusive uint64 prefix in edge
// order, compacted to (edge, prefix) pairs.
// Each thread takes kScanIt consecutive edges; thread sums are scanned
// within the wave by shuffles and across the block's waves in LDS (integer
// sums: the grouping does not change them).
constexpr int kScanIt = 4;
// Cut-point guide of a table with n entries and total Q (n buckets): the
// least bucket b whose first target ceil(b Q / n) reaches p is
// floor((p - 1) n / Q) + 1 (0 for p = 0).  fp64 estimate, then exact
// integer steps: (p - 1) n < 2^63 for tables of up to 2^21 edges.
__device__ __forceinline__ int cut_bucket(uint64_t p, int n, uint64_t Q) {
    if (p == 0) return 0;
    const uint64_t num = (p - 1) * (uint64_t)n;
    uint64_t b = (uint64_t)((double)num / (double)Q);
    while (b > 0 && b * Q > num) --b;
    while ((b + 1) * Q <= num) ++b;
    return (int)b + 1;
}
template <int BS>
__device__ __forceinline__ void edge_scan_body(int E, const float *__restrict__ w, int *__restrict__ out_edge,
        uint64_t *__restrict__ out_prefix, int *__restrict__ out_n, uint64_t *__restrict__ out_Q,
        int *__restrict__ out_guide, int tbl) {
    constexpr int NW = BS / 64;
    const float *wt = w + (size_t)tbl * E;
    int *oe = out_edge + (size_t)tbl * E;
    uint64_t *op = out_prefix + (size_t)tbl * E;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __shared__ uint64_t s_wsum[NW];
    __shared__ int s_wcnt[NW];
    __shared__ float s_wmax[NW];
    float mx = 0.0f;
    for (int e = threadIdx.x; e < E; e += BS) mx = fmaxf(mx, wt[e]);
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0) s_wmax[wave] = mx;
    __syncthreads();
    float wm = 0.0f;
    for (int k = 0; k < NW; ++k) wm = fmaxf(wm, s_wmax[k]);
    uint64_t base = 0;    // running totals, identical in every thread
    int nbase = 0;
    for (int start = 0; start < E; start += BS * kScanIt) {
        const int e0 = start + threadIdx.x * kScanIt;
        uint32_t q[kScanIt];
        uint64_t tsum = 0;
        int tcnt = 0;
        for (int k = 0; k < kScanIt; ++k) {
            q[k] = 0;
            int e = e0 + k;
            if (e < E) {
                float we = wt[e];
                if (we > 0.0f && wm > 0.0f) q[k] = 1u + (uint32_t)floorf((we / wm) * kQScale);
            }
            tsum += q[k];
            tcnt += q[k] > 0;
        }
        uint64_t isum = tsum;
        int icnt = tcnt;
        for (int off = 1; off < 64; off <<= 1) {
            uint64_t vs = __shfl_up(isum, off);
            int vc = __shfl_up(icnt, off);
            if (lane >= off) { isum += vs; icnt += vc; }
        }
        if (lane == 63) { s_wsum[wave] = isum; s_wcnt[wave] = icnt; }
        __syncthreads();
        uint64_t wsum = 0, total = 0;
        int wcnt = 0, tc = 0;
        for (int k = 0; k < NW; ++k) {
            if (k < wave) { wsum += s_wsum[k]; wcnt += s_wcnt[k]; }
            total += s_wsum[k]; tc += s_wcnt[k];
        }
        uint64_t pre = base + wsum + isum - tsum;
        int slot = nbase + wcnt + icnt - tcnt;
        for (int k = 0; k < kScanIt; ++k)
            if (q[k] > 0) { oe[slot] = e0 + k; op[slot] = pre; pre += q[k]; ++slot; }
        base += total;
        nbase += tc;
        __syncthreads();
    }
    if (threadIdx.x == 0) { out_n[tbl] = nbase; out_Q[tbl] = base; }
    // guide[b], b in [0, n]: the entry that target ceil(b Q / n) picks.
    // Entry i holds the buckets from cut_bucket(p_i) up to cut_bucket(p_i+1)
    // (the last entry up to n), so every bucket is written once.
    int *og = out_guide + (size_t)tbl * (E + 1);
    const int n = nbase;
    for (int i = threadIdx.x; i < n; i += BS) {
        const int b0 = cut_bucket(op[i], n, base);
        const int b1 = i + 1 < n ? cut_bucket(op[i + 1], n, base) : n + 1;
        for (int b = b0; b < b1; ++b) og[b] = i;
    }
}
template <int BS>
__global__ __launch_bounds__(BS) void k_edge_scan(int E, const float *__restrict__ w, int *__restrict__ out_edge,
        uint64_t *__restrict__ out_prefix, int *__restrict__ out_n, uint64_t *__restrict__ out_Q,
        int *__restrict__ out_guide) {
    edge_scan_body<BS>(E, w, out_edge, out_prefix, out_n, out_Q, out_guide, blockIdx.x);
}

// Single context: the same tables, each split over kEsChunk-edge chunks so
// that a table is not one block's sequential walk (the batched path runs a
// block per table of every face, which fills the chip).  The outputs are
// edge_scan_body's bit for bit: the maximum and the integer sums are exact,
// and the chunks and their threads keep edge order.
constexpr int kEsPer = 8, kEsChunk = 256 * kEsPer;
__device__ __forceinline__ uint32_t es_quant(float we, float wm) {
    return (we > 0.0f && wm > 0.0f) ? 1u + (uint32_t)floorf((we / wm) * kQScale) : 0u;
}
// per table: the largest weight (non-negative floats order as their bits)
__global__ __launch_bounds__(256) void k_es_max(int E, const float *__restrict__ w, uint32_t *__restrict__ wmax) {
    __shared__ float s_m[4];
    const float *wt = w + (size_t)blockIdx.y * E;
    const int e1 = min(E, (int)(blockIdx.x + 1) * kEsChunk);
    float mx = 0.0f;
    for (int e = blockIdx.x * kEsChunk + threadIdx.x; e < e1; e += 256) mx = fmaxf(mx, wt[e]);
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float m = fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3]));
        if (m > 0.0f) atomicMax(&wmax[blockIdx.y], __float_as_uint(m));
    }
}
// per (table, chunk): the quantised weights' sum and positive count
__global__ __launch_bounds__(256) void k_es_sum(int E, const float *__restrict__ w, const uint32_t *__restrict__ wmax,
        uint64_t *__restrict__ csum, uint32_t *__restrict__ ccnt) {
    __shared__ uint64_t s_s[4];
    __shared__ uint32_t s_c[4];
    const float *wt = w + (size_t)blockIdx.y * E;
    const float wm = __uint_as_float(wmax[blockIdx.y]);
    const int e0 = blockIdx.x * kEsChunk + threadIdx.x * kEsPer;
    uint64_t sum = 0;
    uint32_t cnt = 0;
    for (int k = 0; k < kEsPer; ++k)
        if (e0 + k < E) { const uint32_t q = es_quant(wt[e0 + k], wm); sum += q; cnt += q > 0; }
    for (int off = 32; off > 0; off >>= 1) { sum += __shfl_xor(sum, off); cnt += __shfl_xor(cnt, off); }
    if ((threadIdx.x & 63) == 0) { s_s[threadIdx.x >> 6] = sum; s_c[threadIdx.x >> 6] = cnt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        csum[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s_s[0] + s_s[1] + s_s[2] + s_s[3];
        ccnt[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
    }
}
// per (table, chunk): offsets from the earlier chunks, then the chunk's
// exclusive scan and compaction; the last chunk writes n and Q
__global__ __launch_bounds__(256) void k_es_scan(int E, const float *__restrict__ w,
        const uint32_t *__restrict__ wmax, const uint64_t *__restrict__ csum, const uint32_t *__restrict__ ccnt,
        int *__restrict__ out_edge, uint64_t *__restrict__ out_prefix, int *__restrict__ out_n,
        uint64_t *__restrict__ out_Q) {
    __shared__ uint64_t s_s[4];
    __shared__ uint32_t s_c[4];
    const int tbl = blockIdx.y, nch = gridDim.x, ch = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // offsets: the sums of chunks 0 .. ch-1
    uint64_t b = 0;
    uint32_t nb = 0;
    for (int c = threadIdx.x; c < ch; c += 256) { b += csum[(size_t)tbl * nch + c]; nb += ccnt[(size_t)tbl * nch + c]; }
    for (int off = 32; off > 0; off >>= 1) { b += __shfl_xor(b, off); nb += __shfl_xor(nb, off); }
    if (lane == 0) { s_s[wave] = b; s_c[wave] = nb; }
    __syncthreads();
    const uint64_t base = s_s[0] + s_s[1] + s_s[2] + s_s[3];
    const uint32_t nbase = s_c[0] + s_c[1] + s_c[2] + s_c[3];
    __syncthreads();
    const float *wt = w + (size_t)tbl * E;
    const float wm = __uint_as_float(wmax[tbl]);
    const int e0 = ch * kEsChunk + threadIdx.x * kEsPer;
    uint32_t q[kEsPer];
    uint64_t tsum = 0;
    uint32_t tcnt = 0;
    for (int k = 0; k < kEsPer; ++k) {
        q[k] = e0 + k < E ? es_quant(wt[e0 + k], wm) : 0u;
        tsum += q[k];
        tcnt += q[k] > 0;
    }
    uint64_t isum = tsum;
    uint32_t icnt = tcnt;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t vs = __shfl_up(isum, off);
        const uint32_t vc = __shfl_up(icnt, off);
        if (lane >= off) { isum += vs; icnt += vc; }
    }
    if (lane == 63) { s_s[wave] = isum; s_c[wave] = icnt; }
    __syncthreads();
    uint64_t wsum = 0, total = 0;
    uint32_t wcnt = 0, tc = 0;
    for (int k = 0; k < 4; ++k) {
        if (k < wave) { wsum += s_s[k]; wcnt += s_c[k]; }
        total += s_s[k]; tc += s_c[k];
    }
    uint64_t pre = base + wsum + isum - tsum;
    uint32_t slot = nbase + wcnt + icnt - tcnt;
    int *oe = out_edge + (size_t)tbl * E;
    uint64_t *op = out_prefix + (size_t)tbl * E;
    for (int k = 0; k < kEsPer; ++k)
        if (q[k] > 0) { oe[slot] = e0 + k; op[slot] = pre; pre += q[k]; ++slot; }
    if (ch == nch - 1 && threadIdx.x == 0) { out_n[tbl] = (int)(nbase + tc); out_Q[tbl] = base + total; }
}
// per (table, range of entries): the cut-point guide, as edge_scan_body
__global__ __launch_bounds__(256) void k_es_guide(int E, const uint64_t *__restrict__ out_prefix,
        const int *__restrict__ out_n, const uint64_t *__restrict__ out_Q, int *__restrict__ out_guide) {
    const int tbl = blockIdx.y, n = out_n[tbl];
    const uint64_t Q = out_Q[tbl];
    const uint64_t *op = out_prefix + (size_t)tbl * E;
    int *og = out_guide + (size_t)tbl * (E + 1);
    const int i1 = min(n, (int)(blockIdx.x + 1) * kEsChunk);
    for (int i = blockIdx.x * kEsChunk + threadIdx.x; i < i1; i += 256) {
        const int b0 = cut_bucket(op[i], n, Q);
        const int b1 = i + 1 < n ? cut_bucket(op[i + 1], n, Q) : n + 1;
        for (int bb = b0; bb < b1; ++bb) og[bb] = i;
    }
}

// ------------------------------------------------------ LDS staging -----
__device__ inline void stage_tables(const Scene &S, Light *Ls, float *spec_lds) {
    for (int j = threadIdx.x; j < S.nl; j += blockDim.x) {
        const float *g = S.lgeom + 12 * j;
        Light L;
        L.c = mk(g[0], g[1], g[2]); L.e1 = mk(g[3], g[4], g[5]); L.e2 = mk(g[6], g[7], g[8]);
        L.n = mk(g[9], g[10], g[11]);
        L.area = len(cross(L.e1, L.e2));
        L.r = S.lrgb[3 * j]; L.g = S.lrgb[3 * j + 1]; L.b = S.lrgb[3 * j + 2];
        Ls[j] = L;
    }
    for (int k = threadIdx.x; k < S.res * S.res; k += blockDim.x) spec_lds[k] = S.spec[k];
}

// light j's (u, v) for a sample whose light words start at word 'off'
// (off + 2j, off + 2j + 1) of counters (idx, block, tag, 0)
struct LightRng {
    uint64_t seed; uint32_t idx, tag; int off; int cur; u4 blk;
    __device__ LightRng(uint64_t s, uint32_t i, uint32_t t, int o) : seed(s), idx(i), tag(t), off(o), cur(-1) {}
    __device__ __forceinline__ void get(int j, float &u, float &v) {
        int wi = off + 2 * j, b = wi >> 2;
        if (b != cur) { blk = philox(seed, idx, (uint32_t)b, tag, 0); cur = b; }
        if (wi & 2) { u = u01(blk.z); v = u01(blk.w); } else { u = u01(blk.x); v = u01(blk.y); }
    }
};

// camera sample s: jittered pixel ray
__device__ __forceinline__ v3 camera_sample(const Scene &S, uint64_t seed, uint32_t s, int spp, int &pix) {
    pix = (int)(s / (uint32_t)spp);
    int px = pix % S.W, py = pix / S.W;
    u4 w0 = philox(seed, s, 0, 0, 0);
    return camera_dir(S, (float)px + u01(w0.x), (float)py + u01(w0.y));
}

// counters, 8 per kernel: 0 camera rays, 1 shadow rays, 2 primary-edge rays,
// 3 secondary-edge rays, 4 box tests, 5 triangle tests, 6 shaded light samples.
// Each counter is spread over kCtrSpread copies one 128-byte line apart,
// picked by the wave's index: device-scope atomics to one word serialise
// (about 12 ns apiece here), which held back kernels whose every wave added
// to the same few words.  fr_stats sums the copies.
constexpr int kCtrSpread = 64, kCtrPad = 16;
constexpr int kCtrPerKern = 8 * kCtrSpread * kCtrPad;   // words per kernel
__device__ inline void flush_count(unsigned long long *ctr, int slot, unsigned long long v) {
    unsigned long long s = v;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    const unsigned r = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (kCtrSpread - 1);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(&ctr[(slot * kCtrSpread + r) * kCtrPad], s);
}
__device__ inline void flush_work(unsigned long long *ctr, const Work &w) {
    flush_count(ctr, 4, (unsigned long long)w.box - w.box_back);   // the wave's sum is >= 0
    flush_count(ctr, 5, w.tri);
    flush_count(ctr, 6, w.shade);
}

// ------------------------------------------------ forward wavefront -----
// The forward pass runs in three steps over a chunk of camera samples:
//   camera        jittered pinhole ray, closest hit -> 16-byte hit record
//                 (k_cam_* below; the batched path walks the tree per
//                 sample, fwd_camera_body);
//   shadow rays   per (sample, light): horizon test, shadow ray, one bit
//                 per light in the sample's visibility mask (k_sh_propose
//                 and k_sh_trace below);
//   k_fwd_shade   one lane per sample: shading of the visible lights (no
//                 traversal).
// The adjoint and the shadow-boundary kernels read the same records; when a
// render's samples exceed one chunk the backward recomputes them per chunk.
struct HitRec { int tri; float b1, b2, det; };

__device__ __forceinline__ Hit hit_of(HitRec r) {
    Hit h; h.tri = r.tri; h.t = 0.0f; h.b1 = r.b1; h.b2 = r.b2; h.det = r.det;
    return h;
}

__device__ __forceinline__ void fwd_camera_body(const Scene &S, uint64_t seed, int spp, long long s0, long long n,
        HitRec *__restrict__ hits, unsigned long long *__restrict__ vis, unsigned long long *ctr, int bx) {
    long long i = (long long)bx * blockDim.x + threadIdx.x;
    uint32_t n_cam = 0;
    Work wk;
    if (i < n) {
        int pix;
        v3 o = mk(S.cam_x, S.cam_y, S.cam_z);
        v3 d = camera_sample(S, seed, (uint32_t)(s0 + i), spp, pix);
        Hit h = trace_closest(S, o, d, wk);
        HitRec r; r.tri = h.tri; r.b1 = h.b1; r.b2 = h.b2; r.det = h.det;
        hits[i] = r;
        vis[i] = 0ull;
        n_cam = 1;
    }
    flush_count(ctr, 0, n_cam);
    flush_work(ctr, wk);
}

// Camera rays without the tree.  A camera sample's hit is the minimum of
// (t, triangle id) over the triangles whose ray/triangle test accepts its
// ray: the rule the closest-hit walk applies, so both give the same record
// bit for bit.  An accepted hit point lies in the triangle's box widened by
// the hit margin, so the screen footprint of that box (plus a rounding
// margin) holds every sample the triangle can be hit by.  Three passes over
// a chunk:
//   k_cam_init     the sample's screen position (into its hit record) and an
//                  empty key (into its visibility word);
//   k_cam_raster   one lane per (triangle, sample index within the pixel):
//                  the ray/triangle test for that sample of every pixel of
//                  the footprint, accepted hits folded into the key with a
//                  64-bit atomic min (t > 0 orders like its bit pattern, the
//                  low word is the triangle id, so equal t keeps the lowest);
//   k_cam_resolve  the key back into a hit record (the winner's test run
//                  again for its barycentrics) and a cleared visibility mask.
__global__ __launch_bounds__(256) void k_cam_init(Scene S, uint64_t seed, int spp, long long s0, long long n,
        HitRec *__restrict__ hits, unsigned long long *__restrict__ key) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t s = (uint32_t)(s0 + i);
    const int pix = (int)(s / (uint32_t)spp);
    const int px = pix % S.W, py = pix / S.W;
    const u4 w0 = philox(seed, s, 0, 0, 0);
    HitRec r;
    r.tri = -1; r.b1 = (float)px + u01(w0.x); r.b2 = (float)py + u01(w0.y); r.det = 0.0f;
    hits[i] = r;
    key[i] = ~0ull;
}

// Inclusive pixel range that holds the screen positions of every point of
// the triangle's widened box (the whole image when the box reaches the
// camera's plane).  Projection in fp64; the margin covers the fp32 rounding
// of the sample's direction and of the hit point.
__device__ inline void cam_footprint(const Scene &S, v3 v0, v3 v1, v3 v2, int border, int &x0, int &x1, int &y0,
                                     int &y1) {
    // pixels -border .. W - 1 + border (a border of 1 holds screen points
    // just outside the image)
    const int lx = -border, hx = S.W - 1 + border, ly = -border, hy = S.H - 1 + border;
    x0 = lx; x1 = hx; y0 = ly; y1 = hy;
    const double lo[3] = {(double)fminf(fminf(v0.x, v1.x), v2.x) - 2.0 * kHitMargin,
                          (double)fminf(fminf(v0.y, v1.y), v2.y) - 2.0 * kHitMargin,
                          (double)fminf(fminf(v0.z, v1.z), v2.z) - 2.0 * kHitMargin};
    const double hi[3] = {(double)fmaxf(fmaxf(v0.x, v1.x), v2.x) + 2.0 * kHitMargin,
                          (double)fmaxf(fmaxf(v0.y, v1.y), v2.y) + 2.0 * kHitMargin,
                          (double)fmaxf(fmaxf(v0.z, v1.z), v2.z) + 2.0 * kHitMargin};
    const double cx = S.cam_x, cy = S.cam_y, cz = S.cam_z, ps = S.ps;
    const double dmin = cz - hi[2];                    // the camera looks along -z: depth = t
    const double ext = fmax(fmax(fabs(cx), fabs(cy)), fabs(cz)) +
                       fmax(fmax(fmax(fabs(lo[0]), fabs(hi[0])), fmax(fabs(lo[1]), fabs(hi[1]))),
                            fmax(fabs(lo[2]), fabs(hi[2])));
    if (!(dmin > 1e-4 * (ext + 1.0))) return;         // reaches the camera's plane: every pixel
    // fp32 error of the hit point (a few ulp of its magnitude) seen through
    // the projection, plus that of the sample's direction, with room to spare
    const double sc_far = 1.0 / ((cz - lo[2]) * ps), sc_near = 1.0 / (dmin * ps);   // pixels per metre
    const double eps = 0.125 + 8.0 * 1.2e-7 * ext * sc_near + 8.0 * 1.2e-7 * (double)max(S.W, S.H);
    double qx0 = 1e300, qx1 = -1e300, qy0 = 1e300, qy1 = -1e300;
    for (int k = 0; k < 8; ++k) {
        const double x = (k & 1) ? hi[0] : lo[0], y = (k & 2) ? hi[1] : lo[1];
        const double sc = (k & 4) ? sc_near : sc_far;
        const double qx = 0.5 * S.W + (x - cx) * sc, qy = 0.5 * S.H - (y - cy) * sc;
        qx0 = fmin(qx0, qx); qx1 = fmax(qx1, qx); qy0 = fmin(qy0, qy); qy1 = fmax(qy1, qy);
    }
    // clamped before the conversion (an off-screen box gives an empty range)
    x0 = (int)fmin(fmax((double)lx, floor(qx0 - eps)), (double)(hx + 1));
    x1 = (int)fmax(fmin((double)hx, floor(qx1 + eps)), (double)(lx - 1));
    y0 = (int)fmin(fmax((double)ly, floor(qy0 - eps)), (double)(hy + 1));
    y1 = (int)fmax(fmin((double)hy, floor(qy1 + eps)), (double)(ly - 1));
}

__global__ __launch_bounds__(256) void k_cam_raster(Scene S, int spp, long long s0, long long n,
        const HitRec *__restrict__ hits, unsigned long long *__restrict__ key, unsigned long long *ctr) {
    const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
    uint32_t n_tri = 0;
    if (g < (long long)S.F * spp) {
        const int f = (int)(g / spp), k = (int)(g % spp);
        const int *t = S.faces + 3 * f;
        const v3 v0 = vpos(S, t[0]), v1 = vpos(S, t[1]), v2 = vpos(S, t[2]);
        int x0, x1, y0, y1;
        cam_footprint(S, v0, v1, v2, 0, x0, x1, y0, y1);
        // rows of this chunk
        y0 = max(y0, (int)((s0 / spp) / S.W));
        y1 = min(y1, (int)(((s0 + n - 1) / spp) / S.W));
        const v3 o = mk(S.cam_x, S.cam_y, S.cam_z);
        for (int py = y0; py <= y1; ++py)
            for (int px = x0; px <= x1; ++px) {
                const long long i = ((long long)py * S.W + px) * spp + k - s0;
                if (i < 0 || i >= n) continue;
                const HitRec q = hits[i];
                const v3 d = camera_dir(S, q.b1, q.b2);
                float tt, b1, b2, det;
                ++n_tri;
                if (ray_tri(o, d, v0, v1, v2, 0.0f, INFINITY, tt, b1, b2, det))
                    atomicMin(&key[i], ((unsigned long long)__float_as_uint(tt) << 32) | (unsigned)f);
            }
    }
    flush_count(ctr, 5, n_tri);
}

__global__ __launch_bounds__(256) void k_cam_resolve(Scene S, long long n, HitRec *__restrict__ hits,
        unsigned long long *__restrict__ vis, unsigned long long *ctr) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    uint32_t n_cam = 0;
    if (i < n) {
        const unsigned long long kv = vis[i];
        HitRec r = hits[i];
        const v3 d = camera_dir(S, r.b1, r.b2);
        r.tri = -1; r.b1 = r.b2 = r.det = 0.0f;
        if (kv != ~0ull) {
            const int f = (int)(uint32_t)kv;
            const int *t = S.faces + 3 * f;
            float tt, b1, b2, det;
            if (ray_tri(mk(S.cam_x, S.cam_y, S.cam_z), d, vpos(S, t[0]), vpos(S, t[1]), vpos(S, t[2]), 0.0f,
                        INFINITY, tt, b1, b2, det)) {
                r.tri = f; r.b1 = b1; r.b2 = b2; r.det = det;
            }
        }
        hits[i] = r;
        vis[i] = 0ull;
        n_cam = 1;
    }
    flush_count(ctr, 0, n_cam);
}

// Rays are compacted before they are traced: the lanes run the horizon
// tests and append the rays that need tracing to lists (one LDS atomic per
// wave and list).  About a third of the (sample, light) pairs need a ray at
// the paper's framing (camera misses and lights below the horizon need
// none), so tracing in place would leave two lanes in three idle.  The
// shadow-boundary kernel takes a tile of samples for one light per block;
// the tile size is a template parameter of its body (the batched launcher
// may pick 256 or 512); its default tile is 256 samples.
constexpr int kSecTile = 256;
__device__ __forceinline__ int lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// Single context: the shadow rays in two kernels.  After a fused block's
// compaction only about a third of its lanes have a ray (most pairs fail
// the horizon test), so most of its waves sit idle while the rest trace.
//   k_sh_propose  one block per 256 samples for all lights: each sample's
//                 surface decided once, then every light's horizon test;
//                 the accepted samples' indices go to each light's queue
//                 (one atomic per block and light on that light's counter);
//   k_sh_trace    one lane per queued ray, rebuilt from the sample's hit
//                 record and light sample as k_sh_propose built it, traced.
// Every resident wave of k_sh_trace traces.  The batched path runs the same
// bodies.
__device__ __forceinline__ bool sh_ray(const Scene &S, const Light &L, uint64_t seed, long long s0, long long i,
                                       const HitRec *__restrict__ hits, int j, v3 &p, v3 &dd, int &tri) {
    const HitRec rec = hits[i];
    if (rec.tri < 0) return false;
    const Hit h = hit_of(rec);
    SurfDec sd;
    surf_decide(S, mk(S.cam_x, S.cam_y, S.cam_z), h, sd);
    LightRng rng(seed, (uint32_t)(s0 + i), 0, 2);
    float u, v;
    rng.get(j, u, v);
    const v3 y = light_point(L, u, v);
    if (!above(sd, y)) return false;
    p = sd.p; dd = y - sd.p; tri = h.tri;
    return true;
}
__device__ __forceinline__ Light light_geom(const Scene &S, int j) {
    const float *g = S.lgeom + 12 * j;
    Light L;
    L.c = mk(g[0], g[1], g[2]); L.e1 = mk(g[3], g[4], g[5]); L.e2 = mk(g[6], g[7], g[8]);
    return L;
}
// The proposals of one block of 256 items (samples or sides) for every
// light: accept(j, L) is this lane's horizon test for light j (its surface
// already decided by the caller).  A light's accepted lanes gather in the
// block's byte list for that light; each list goes to the light's queue
// (row j of a [nl][qcap] array) with one atomic on cnt[j], as the values v
// of its lanes.  Returns how many lights this lane's item was queued for.
template <class Accept>
__device__ __forceinline__ uint32_t propose_all_body(const Scene &S, uint32_t v, uint32_t *__restrict__ queue,
                                                     uint32_t qcap, uint32_t *__restrict__ cnt, Accept accept) {
    __shared__ uint8_t ql[kMaxLights * 256];
    __shared__ uint32_t val[256];
    __shared__ Light Ls[kMaxLights];
    __shared__ int q_n[kMaxLights];
    __shared__ uint32_t q_base[kMaxLights];
    for (int k = threadIdx.x; k < S.nl; k += 256) { Ls[k] = light_geom(S, k); q_n[k] = 0; }
    val[threadIdx.x] = v;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    uint32_t taken = 0;
    for (int j = 0; j < S.nl; ++j) {
        const bool need = accept(j, Ls[j]);
        const unsigned long long m = __ballot(need);
        if (m) {   // the same for every lane of the wave
            int wbase = 0;
            if (lane == 0) wbase = atomicAdd(&q_n[j], __popcll(m));
            wbase = __shfl(wbase, 0);
            if (need) { ql[j * 256 + wbase + lanes_below(m)] = (uint8_t)threadIdx.x; ++taken; }
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < S.nl; j += 256) q_base[j] = q_n[j] > 0 ? atomicAdd(&cnt[j], (uint32_t)q_n[j]) : 0u;
    __syncthreads();
    for (int j = 0; j < S.nl; ++j)
        for (int e = threadIdx.x; e < q_n[j]; e += 256) queue[(size_t)j * qcap + q_base[j] + e] = val[ql[j * 256 + e]];
    return taken;
}
// k_sh_propose: one block per 256 samples for every light.  Each sample's
// surface is decided once, then each light's horizon test runs on the same
// lanes (the decisions of sh_ray).  The batched path runs the same body.
__device__ __forceinline__ void sh_propose_all_body(const Scene &S, uint64_t seed, long long s0, long long n,
        const HitRec *__restrict__ hits, uint32_t *__restrict__ queue, uint32_t qcap, uint32_t *__restrict__ cnt,
        unsigned long long *ctr, int bx) {
    const long long i = (long long)bx * 256 + threadIdx.x;
    bool have = false;
    SurfDec sd;
    if (i < n) {
        const HitRec rec = hits[i];
        if (rec.tri >= 0) {
            surf_decide(S, mk(S.cam_x, S.cam_y, S.cam_z), hit_of(rec), sd);
            have = true;
        }
    }
    LightRng rng(seed, (uint32_t)(s0 + i), 0, 2);
    const uint32_t n_sh = propose_all_body(S, (uint32_t)i, queue, qcap, cnt, [&](int j, const Light &L) {
        if (!have) return false;
        float u, v;
        rng.get(j, u, v);
        return above(sd, light_point(L, u, v));
    });
    flush_count(ctr, 1, n_sh);
}
__global__ __launch_bounds__(256) void k_sh_propose(Scene S, uint64_t seed, long long s0, long long n,
        const HitRec *__restrict__ hits, uint32_t *__restrict__ queue, uint32_t qcap, uint32_t *__restrict__ cnt,
        unsigned long long *ctr) {
    sh_propose_all_body(S, seed, s0, n, hits, queue, qcap, cnt, ctr, blockIdx.x);
}
// k_sh_trace runs one wave per block (both paths), k_pv_trace takes its block
// size from the launch.  One wave per block: a wave whose rays have
// all ended frees its slot at once, where a wave of a four-wave block holds
// the block's place until the other three end too (1.40 -> 1.34 ms at paper
// scale; 128-thread blocks 1.37).  k_pv_trace runs the same way (with the
// queued triangle tests and the adjoint on three streams, the step went
// from 3.02 to 2.98 ms; 128-thread blocks 3.00).
constexpr int kTraceBlock = 64;
__device__ __forceinline__ void sh_trace_body(const Scene &S, uint64_t seed, long long s0,
        const HitRec *__restrict__ hits, const uint32_t *__restrict__ queue, uint32_t qcap,
        const uint32_t *__restrict__ cnt, unsigned long long *__restrict__ vis, unsigned long long *ctr, int bx,
        int j) {
    static_assert(kTraceBlock == 64, "one wave per block: the walk's test list is the block's");
    __shared__ uint32_t lq[2 * kLeafList + 64];            // the wave's list of triangle tests
    const uint32_t e = bx * kTraceBlock + threadIdx.x;
    if ((uint32_t)bx * kTraceBlock >= cnt[j]) return;   // the whole block is past the queue
    Work wk;
    if (e < cnt[j]) {
        const uint32_t i = queue[(size_t)j * qcap + e];
        v3 p, dd;
        int tri;
        if (sh_ray(S, light_geom(S, j), seed, s0, i, hits, j, p, dd, tri) &&
            !trace_any(S, p, dd, tri, wk, lq))
            atomicOr(&vis[i], 1ull << j);
    }
    flush_work(ctr, wk);
}
__global__ __launch_bounds__(kTraceBlock) void k_sh_trace(Scene S, uint64_t seed, long long s0,
        const HitRec *__restrict__ hits, const uint32_t *__restrict__ queue, uint32_t qcap,
        const uint32_t *__restrict__ cnt, unsigned long long *__restrict__ vis, unsigned long long *ctr) {
    sh_trace_body(S, seed, s0, hits, queue, qcap, cnt, vis, ctr, blockIdx.x, blockIdx.y);
}

__device__ __forceinline__ void fwd_shade_body(const Scene &S, uint64_t seed, int spp, long long s0, long long n,
        const HitRec *__restrict__ hits, const unsigned long long *__restrict__ vis,
        float *__restrict__ samples, unsigned long long *ctr, int bx) {
    extern __shared__ float dyn[];
    __shared__ Light Ls[kMaxLights];
    float *spec_lds = dyn;
    stage_tables(S, Ls, spec_lds);
    __syncthreads();
    long long i = (long long)bx * blockDim.x + threadIdx.x;
    Work wk;
    if (i < n) {
        HitRec rec = hits[i];
        float c[3] = {0.0f, 0.0f, 0.0f};
        if (rec.tri >= 0) {
            Hit h = hit_of(rec);
            uint32_t s = (uint32_t)(s0 + i);
            int pix;
            v3 o = mk(S.cam_x, S.cam_y, S.cam_z);
            v3 d = camera_sample(S, seed, s, spp, pix);
            unsigned long long m = vis[i];
            SurfDec sd;
            surf_decide(S, o, h, sd);
            Surf<float> sv;
            surf_value<float>(S, spec_lds, o, d, h, sd, sv);
            LightRng rng(seed, s, 0, 2);
            while (m) {
                int j = __ffsll((long long)m) - 1;
                m &= m - 1;
                float u, v;
                rng.get(j, u, v);
                const Light &L = Ls[j];
                v3 y = light_point(L, u, v);
                float cj[3];
                shade_light<float>(sv, L, cvt<float>(y), light_branch(sd, L.n, y), nullptr, cj, nullptr);
                ++wk.shade;
                c[0] += cj[0]; c[1] += cj[1]; c[2] += cj[2];
            }
        }
        samples[3 * (s0 + i)] = c[0]; samples[3 * (s0 + i) + 1] = c[1]; samples[3 * (s0 + i) + 2] = c[2];
    }
    flush_work(ctr, wk);
}
__global__ __launch_bounds__(256) void k_fwd_shade(Scene S, uint64_t seed, int spp, long long s0, long long n,
        const HitRec *__restrict__ hits, const unsigned long long *__restrict__ vis,
        float *__restrict__ samples, unsigned long long *ctr) {
    fwd_shade_body(S, seed, spp, s0, n, hits, vis, samples, ctr, blockIdx.x);
}

__device__ __forceinline__ void pixel_mean_body(int npix, int spp, const float *__restrict__ samples,
                                                float *__restrict__ img, int bx) {
    int p = bx * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    const float *q = samples + (size_t)3 * p * spp;
    for (int k = 0; k < spp; ++k) { a0 += q[3 * k]; a1 += q[3 * k + 1]; a2 += q[3 * k + 2]; }
    float inv = (float)spp;
    img[3 * p] = a0 / inv; img[3 * p + 1] = a1 / inv; img[3 * p + 2] = a2 / inv;
}
__global__ __launch_bounds__(256) void k_pixel_mean(int npix, int spp, const float *__restrict__ samples, float *__restrict__ img) {
    pixel_mean_body(npix, spp, samples, img, blockIdx.x);
}

// ------------------------------------------------------------ adjoint ---
struct GradBufs {
    double *d_light;  // [nl*3]
    double *d_spec;   // [res^2]
    double *d_pos;    // [3V] (interior + edges, before the normal chain)
    double *d_nrm;    // [3V]
    double *d_alb;    // [3V]
};

// Gradient sums use fp64 hardware atomics (buffers are coarse-grained
// device memory), which keeps the summation-order noise far below fp32.
__device__ __forceinline__ void gadd(double *a, double v) { unsafeAtomicAdd(a, v); }
template <class T> __device__ __forceinline__ void atomic_v(double *a, int V, int i, vec3<T> g) {
    gadd(&a[i], (double)g.x); gadd(&a[V + i], (double)g.y); gadd(&a[2 * V + i], (double)g.z);
}

// Chain the adjoints of the shading point p and of the interpolation
// barycentrics into the hit triangle's vertices, with the camera ray fixed.
// p = o + t d moves only along the ray: dt/dv_k = b_k N / (N . d), N = e1 x e2.
// The barycentrics follow v0 + b1 e1 + b2 e2 = o + t d:
// d(b1, b2) -> z = -(g1 (d x e2) + g2 (e1 x d)) / det, dv_k += b_k z.
// Vertex k of the hit triangle receives u * b_k.
template <class T>
__device__ __forceinline__ vec3<T> chain_u(const Surf<T> &s, vec3<T> gp, T gb0, T gb1, T gb2) {
    T gt = dot(gp, s.dir) / s.ndotd;
    T g1 = gb1 - gb0, g2 = gb2 - gb0;
    vec3<T> z = (s.pv * g1 + s.e1xd * g2) * ((T)-1 / s.det);
    return s.N * gt + z;
}
template <class T>
__device__ inline void chain_hit(int V, const Surf<T> &s, vec3<T> gp, T gb0, T gb1, T gb2, double *d_pos) {
    vec3<T> u = chain_u(s, gp, gb0, gb1, gb2);
    for (int k = 0; k < 3; ++k) atomic_v(d_pos, V, s.i[k], u * s.b[k]);
}

// Per-block vertex accumulator in LDS: the adjoints of a vertex's position,
// normal and albedo (9 values) from all the block's samples are summed in
// fp64 LDS atomics and leave the block as one set of global atomics.  The
// block's 256 samples span a few pixels, so they touch a few dozen
// vertices; a vertex that finds no slot within kVtxProbe probes goes
// straight to the global buffers.
constexpr int kVtxSlots = 512;
constexpr int kVtxProbe = 8;
struct VtxAcc { int *key; double *val; };   // key [slots], val [9][slots]
__device__ __forceinline__ int vtx_slot(const VtxAcc &a, int v) {
    uint32_t h = ((uint32_t)v * 2654435761u) >> 23;     // 9 bits
    for (int p = 0; p < kVtxProbe; ++p) {
        int s = (int)((h + (uint32_t)p) & (kVtxSlots - 1));
        int k = atomicCAS(&a.key[s], -1, v);
        if (k == -1 || k == v) return s;
    }
    return -1;
}
// add (pos, nrm, alb) adjoints of vertex v
template <class T>
__device__ __forceinline__ void vtx_add(const VtxAcc &a, const GradBufs &G, int V, int v, vec3<T> gpos, vec3<T> gnrm,
                                        const T galb[3]) {
    int s = vtx_slot(a, v);
    if (s < 0) {
        atomic_v(G.d_pos, V, v, gpos);
        atomic_v(G.d_nrm, V, v, gnrm);
        for (int c = 0; c < 3; ++c) gadd(&G.d_alb[c * V + v], (double)galb[c]);
        return;
    }
    double x[9] = {(double)gpos.x, (double)gpos.y, (double)gpos.z, (double)gnrm.x, (double)gnrm.y, (double)gnrm.z,
                   (double)galb[0], (double)galb[1], (double)galb[2]};
    for (int c = 0; c < 9; ++c) atomicAdd(&a.val[c * kVtxSlots + s], x[c]);
}
__device__ inline void vtx_clear(const VtxAcc &a) {
    for (int k = threadIdx.x; k < kVtxSlots; k += blockDim.x) a.key[k] = -1;
    for (int k = threadIdx.x; k < 9 * kVtxSlots; k += blockDim.x) a.val[k] = 0.0;
}
__device__ inline void vtx_flush(const VtxAcc &a, const GradBufs &G, int V) {
    for (int s = threadIdx.x; s < kVtxSlots; s += blockDim.x) {
        int v = a.key[s];
        if (v < 0) continue;
        double *dst[3] = {G.d_pos, G.d_nrm, G.d_alb};
        for (int c = 0; c < 9; ++c) {
            double x = a.val[c * kVtxSlots + s];
            if (x != 0.0) gadd(&dst[c / 3][(c % 3) * V + v], x);
        }
    }
}

// The block's light sums have kLightCopies copies, a lane adding into copy
// (lane mod kLightCopies): the lanes of a wave add to the same few words,
// and LDS atomics to one word serialise.  The copies lie an odd number of
// words apart (light_stride), so a word's copies fall in different banks;
// the flush sums them.
constexpr int kLightCopies = 8;
__host__ __device__ __forceinline__ int light_stride(int nl) { return 3 * nl | 1; }
// Interior adjoint of one camera sample (decisions fp32, values T).
// Light and texel adjoints go to block-shared fp32 accumulators when given,
// else straight to the fp64 buffers.
template <class T>
__device__ inline void adjoint_sample(const Scene &S, const Light *Ls, uint64_t seed, uint32_t s,
                                      const float *wf, const Hit &h, const SurfDec &sd, const Surf<T> &sv,
                                      float *g_light_lds, float *g_spec_lds, const VtxAcc &acc,
                                      const GradBufs &G, unsigned long long vis, Work &wk) {
    int V = S.V;
    T w[3] = {(T)wf[0], (T)wf[1], (T)wf[2]};
    vec3<T> gp = vk<T>(0, 0, 0), gns = vk<T>(0, 0, 0), gwo = vk<T>(0, 0, 0);
    T gA[3] = {0, 0, 0}, gks = 0;
    LightRng rng(seed, s, 0, 2);
    while (vis) {               // the forward pass's visibility decisions
        int j = __ffsll((long long)vis) - 1;
        vis &= vis - 1;
        float u, v;
        rng.get(j, u, v);
        const Light &L = Ls[j];
        v3 y = light_point(L, u, v);
        T c[3];
        LAdj<T> a;
        shade_light<T>(sv, L, cvt<T>(y), light_branch(sd, L.n, y), w, c, &a);
        ++wk.shade;
        for (int k = 0; k < 3; ++k) {
            if (g_light_lds)   // this lane's copy of the block's light sums
                atomicAdd(&g_light_lds[(threadIdx.x & (kLightCopies - 1)) * light_stride(S.nl) + 3 * j + k],
                          (float)a.gl[k]);
            else gadd(&G.d_light[3 * j + k], (double)a.gl[k]);
            gA[k] += a.gA[k];
        }
        gks += a.gks;
        gp = gp + a.gp; gns = gns + a.gns; gwo = gwo + a.gwo;
    }
    T gb[3] = {0, 0, 0};
    if (gks != (T)0)
        for (int k = 0; k < 4; ++k) {
            if (g_spec_lds) atomicAdd(&g_spec_lds[sv.tex[k]], (float)(gks * sv.tw[k]));
            else gadd(&G.d_spec[sv.tex[k]], (double)(gks * sv.tw[k]));
        }
    T guvx = gks * sv.dks_du, guvy = gks * sv.dks_dv;
    for (int k = 0; k < 3; ++k) {
        int vi = sv.i[k];
        gb[k] += guvx * (T)S.uv[vi] + guvy * (T)S.uv[V + vi];
        for (int c = 0; c < 3; ++c) gb[k] += gA[c] * (T)S.alb[c * V + vi];
    }
    gp = gp - norm_adj(gwo, sv.wo, sv.olen);
    vec3<T> nt = sv.nu * ((T)1 / sv.nlen);
    vec3<T> gnu = norm_adj(gns * sv.sg, nt, sv.nlen);
    for (int k = 0; k < 3; ++k) {
        int vi = sv.i[k];
        gb[k] += dot(vk<T>((T)S.nrm[vi], (T)S.nrm[V + vi], (T)S.nrm[2 * V + vi]), gnu);
    }
    vec3<T> u = chain_u(sv, gp, gb[0], gb[1], gb[2]);
    for (int k = 0; k < 3; ++k) {
        T ga[3] = {sv.b[k] * gA[0], sv.b[k] * gA[1], sv.b[k] * gA[2]};
        vtx_add<T>(acc, G, V, sv.i[k], u * sv.b[k], gnu * sv.b[k], ga);
    }
}

// Interior adjoint, fp32: one lane per camera sample of the chunk, reading
// the sample's hit record and visibility mask.
__device__ __forceinline__ void render_adj_body(const Scene &S, uint64_t seed, int spp, long long s0, long long n,
        const float *__restrict__ dLdI, const GradBufs &G, const HitRec *__restrict__ hits,
        const unsigned long long *__restrict__ vis, unsigned long long *ctr, int bx) {
    extern __shared__ float dyn[];
    __shared__ Light Ls[kMaxLights];
    float *spec_lds = dyn;
    float *g_spec = dyn + S.res * S.res;        // [res^2]
    float *g_light = g_spec + S.res * S.res;    // [kLightCopies][light_stride(nl)]
    __shared__ int vt_key[kVtxSlots];
    __shared__ double vt_val[9 * kVtxSlots];
    const VtxAcc acc{vt_key, vt_val};
    stage_tables(S, Ls, spec_lds);
    for (int k = threadIdx.x; k < S.res * S.res; k += blockDim.x) g_spec[k] = 0.0f;
    for (int k = threadIdx.x; k < kLightCopies * light_stride(S.nl); k += blockDim.x) g_light[k] = 0.0f;
    vtx_clear(acc);
    __syncthreads();
    long long i = (long long)bx * blockDim.x + threadIdx.x;
    Work wk;
    if (i < n) {
        HitRec rec = hits[i];
        uint32_t s = (uint32_t)(s0 + i);
        int pix;
        v3 o = mk(S.cam_x, S.cam_y, S.cam_z);
        v3 d = camera_sample(S, seed, s, spp, pix);
        float inv = 1.0f / (float)spp;
        float w[3] = {dLdI[3 * pix] * inv, dLdI[3 * pix + 1] * inv, dLdI[3 * pix + 2] * inv};
        if (rec.tri >= 0 && (w[0] != 0.0f || w[1] != 0.0f || w[2] != 0.0f)) {
            Hit h = hit_of(rec);
            SurfDec sd;
            surf_decide(S, o, h, sd);
            Surf<float> sv;
            surf_value<float>(S, spec_lds, o, d, h, sd, sv);
            adjoint_sample<float>(S, Ls, seed, s, w, h, sd, sv, g_light, g_spec, acc, G, vis[i], wk);
        }
    }
    flush_work(ctr, wk);
    __syncthreads();
    for (int k = threadIdx.x; k < S.res * S.res; k += blockDim.x)
        if (g_spec[k] != 0.0f) gadd(&G.d_spec[k], (double)g_spec[k]);
    for (int k = threadIdx.x; k < 3 * S.nl; k += blockDim.x) {
        float x = 0.0f;
        for (int r = 0; r < kLightCopies; ++r) x += g_light[r * light_stride(S.nl) + k];
        if (x != 0.0f) gadd(&G.d_light[k], (double)x);
    }
    vtx_flush(acc, G, S.V);
}
__global__ __launch_bounds__(256) void k_render_adj(Scene S, uint64_t seed, int spp, long long s0, long long n,
        const float *__restrict__ dLdI, GradBufs G, const HitRec *__restrict__ hits,
        const unsigned long long *__restrict__ vis, unsigned long long *ctr) {
    render_adj_body(S, seed, spp, s0, n, dLdI, G, hits, vis, ctr, blockIdx.x);
}

#ifndef FR_EDGE_REAL
#define FR_EDGE_REAL double
#endif
using ER = FR_EDGE_REAL;   // value type of the edge samples
using e3 = vec3<ER>;

// Shadow-boundary (secondary) edge sample of light j at a camera sample's
// shading point; decisions fp32, values in ER.
// The shadow-boundary sample of light j at one camera sample, in one of
// three modes that share the decisions:
//   kSecPropose  stops before the two shadow rays; true when the sample
//                needs them;
//   kSecTrace    traces them; true when they disagree (the sample then has
//                a value), vp = whether the + side sees the light;
//   kSecValue    takes vp as given and scatters the sample's value.
enum { kSecPropose, kSecTrace, kSecValue };
template <int kMode>
__device__ inline bool secondary_edge(const Scene &S, const Light &L, int j, uint64_t seed, uint32_t sidx,
                                      const float *spec_lds, v3 o, v3 dcam, const Hit &h, const SurfDec &sf,
                                      const float *w, double *d_pos, bool &vp, uint32_t &n_rays, Work &steps,
                                      float geoR, v3 *d_sides = nullptr) {
    int n = S.se_n[j];
    uint64_t Q = S.se_Q[j];
    if (n == 0 || Q == 0) return false;
    u4 wd = philox(seed, sidx, (uint32_t)j, 1, 0);
    const uint64_t *pre = S.se_prefix + (size_t)j * S.E;
    uint64_t target = __umul64hi(((uint64_t)wd.y << 32) | wd.x, Q);
    int i = cdf_pick_guided(pre, S.se_guide + (size_t)j * (S.E + 1), n, Q, target);
    int e = S.se_edge[(size_t)j * S.E + i];
    {   // the plane pre-test (edge_weights_body): most proposals end here
        const float4 q1 = S.edge_pl[2 * (size_t)e], q2 = S.edge_pl[2 * (size_t)e + 1];
        const v3 p = sf.p;
        const float t1 = dot(mk(q1.x, q1.y, q1.z), p) - q1.w, t2 = dot(mk(q2.x, q2.y, q2.z), p) - q2.w;
        const float eps = 5.9604645e-8f;
        const float base = 64.0f * eps * (fmaxf(fmaxf(fabsf(p.x), fabsf(p.y)), fabsf(p.z)) + geoR);
        const float b1 = base + 4.0f * eps * fabsf(t1), b2 = base + 4.0f * eps * fabsf(t2);
        if ((t1 > b1 && t2 > b2) || (t1 < -b1 && t2 < -b2)) return false;
    }
    // the edge's endpoints, its faces' normals and first vertices (the
    // values face_normal and vpos give), and the face ids
    const float4 *er = S.edge_rec + 5 * (size_t)e;
    const float4 r0 = er[0], r1 = er[1], r2 = er[2], r3 = er[3], r4 = er[4];
    const int f1 = __float_as_int(r4.z), f2 = __float_as_int(r4.w);
    if (f1 == h.tri || f2 == h.tri) return false;
    v3 p = sf.p;
    if (f2 >= 0) {
        float s1 = dot(mk(r1.z, r1.w, r2.x), p - mk(r2.y, r2.z, r2.w));
        float s2 = dot(mk(r3.x, r3.y, r3.z), p - mk(r3.w, r4.x, r4.y));
        if ((s1 > 0.0f) == (s2 > 0.0f)) return false;
    }
    float tu = u01(wd.z);
    v3 a = mk(r0.x, r0.y, r0.z), b = mk(r0.w, r1.x, r1.y);
    v3 sp = mk(a.x + tu * (b.x - a.x), a.y + tu * (b.y - a.y), a.z + tu * (b.z - a.z));
    float den = dot(L.n, sp - p);
    if (den == 0.0f) return false;
    float lam = dot(L.n, L.c - p) / den;
    if (!(lam > 1.0f)) return false;
    v3 y = mk(p.x + lam * (sp.x - p.x), p.y + lam * (sp.y - p.y), p.z + lam * (sp.z - p.z));
    v3 ql = y - L.c;
    if (!(fabsf(dot(ql, L.e1)) <= 0.5f * dot(L.e1, L.e1) && fabsf(dot(ql, L.e2)) <= 0.5f * dot(L.e2, L.e2))) return false;
    if (!above(sf, y)) return false;
    v3 m = cross(a - p, b - p);
    float mn = dot(m, L.n);
    v3 mp = mk(m.x - mn * L.n.x, m.y - mn * L.n.y, m.z - mn * L.n.z);
    float lm = sqrtf(dot(mp, mp));
    if (lm == 0.0f) return false;
    v3 un = mk(mp.x / lm, mp.y / lm, mp.z / lm);
    v3 yp = mk(y.x + kEdgeOffM * un.x, y.y + kEdgeOffM * un.y, y.z + kEdgeOffM * un.z);
    v3 ym = mk(y.x - kEdgeOffM * un.x, y.y - kEdgeOffM * un.y, y.z - kEdgeOffM * un.z);
    if (kMode == kSecPropose) {
        if (d_sides) { d_sides[0] = yp - p; d_sides[1] = ym - p; }
        return true;
    }
    if (kMode == kSecTrace) {
        n_rays += 2;
        bool bp, bm;
        trace_any2(S, p, yp - p, ym - p, h.tri, bp, bm, steps);
        vp = !bp;
        return bp != bm;
    }
    // ---- value path
    Surf<ER> sd;
    surf_value<ER>(S, spec_lds, o, dcam, h, sf, sd);
    ER hc[3];
    shade_light<ER>(sd, L, cvt<ER>(y), light_branch(sf, L.n, y), nullptr, hc, nullptr);
    ER hw = ((ER)w[0] * hc[0] + (ER)w[1] * hc[1] + (ER)w[2] * hc[2]) / (ER)L.area;
    e3 P = sd.p, A = cvt<ER>(a), B = cvt<ER>(b), Y = cvt<ER>(y), Nl = cvt<ER>(L.n);
    e3 pa = A - P, pb = B - P, py = Y - P;
    e3 mval = cross(pa, pb);
    e3 dpsi_a = cross(pb, py), dpsi_b = cross(py, pa);
    e3 dpsi_p = (mval + dpsi_a + dpsi_b) * (ER)-1;
    e3 bma = B - A;
    e3 Sd = A + bma * (ER)tu;
    ER nsp = dot(Nl, Sd - P);
    ER lamd = dot(Nl, cvt<ER>(L.c) - P) / nsp;
    e3 dydt = bma * lamd - (Sd - P) * (lamd * dot(Nl, bma) / nsp);
    e3 mpar = mval - Nl * dot(mval, Nl);
    uint64_t qe = (i + 1 < n ? pre[i + 1] : Q) - pre[i];
    ER pe = (ER)((double)qe / (double)Q);
    ER W = hw * (vp ? (ER)1 : (ER)-1) * len(dydt) / (len(mpar) * pe);
    const int *ed = S.edges + 4 * e;
    atomic_v(d_pos, S.V, ed[0], dpsi_a * W);
    atomic_v(d_pos, S.V, ed[1], dpsi_b * W);
    // the receiver point p moves along the fixed camera ray
    chain_hit<ER>(S.V, sd, dpsi_p * W, (ER)0, (ER)0, (ER)0, d_pos);
    return true;
}

// One block per tile of kSecTile camera samples and group of kSecLights
// lights.  Each
// lane decides its sample's surface once (sec_setup), then runs the edge
// pick and acceptance tests (no rays) for one light after another; the
// first kept the block per (tile, light) and repeated the sample's camera
// ray, hit record and surface for each light, a chain of dependent loads
// ahead of each pick.  A proposal that needs its two side rays goes to the
// block's list in LDS (4 bytes: the list holds every (sample, light) pair of
// the block at worst), and after the proposals the block's waves trace the
// listed pairs' rays.  Proposals are accepted rarely (about 1 in 10^4 at the
// paper's framing), so a listed pair's lane sets up its sample and pick
// again rather than keep the rays: the proposal loop then needs 45 vector
// registers, and the trace phase's registers are not held beside them.
__device__ __forceinline__ void sec_setup(const Scene &S, uint64_t seed, int spp, long long s0, long long i,
        const float *dLdI, const HitRec *hits, v3 &o, v3 &d, float w[3], Hit &h, SurfDec &sd, uint32_t &s,
        bool &live) {
    HitRec rec = hits[i];
    s = (uint32_t)(s0 + i);
    int pix;
    o = mk(S.cam_x, S.cam_y, S.cam_z);
    d = camera_sample(S, seed, s, spp, pix);
    float inv = 1.0f / (float)spp;
    w[0] = dLdI[3 * pix] * inv; w[1] = dLdI[3 * pix + 1] * inv; w[2] = dLdI[3 * pix + 2] * inv;
    live = rec.tri >= 0 && (w[0] != 0.0f || w[1] != 0.0f || w[2] != 0.0f);
    if (live) {
        h = hit_of(rec);
        surf_decide(S, o, h, sd);
    }
}

// k_edge_secondary: decisions and the two shadow rays of each accepted
// sample (compacted per block as above); the samples whose rays disagree
// go to a global list as (chunk index | light << 24 | vp << 30).
// k_edge_secondary_value: the value path of each listed sample.  Splitting
// them keeps the fp64 value code's registers out of the traversal kernel.
// Lights per block, measured at the paper's framing (20 lights; ms per
// step): 1 2.65, 2 2.56, 4 2.44, 5 2.43, 7 2.45, 10 2.48, all 20 2.63 (long
// blocks hold their registers and LDS beside the other two terms for the
// whole adjoint).  The per-(tile, light) form that kept each listed
// proposal's rays took 2.49.
constexpr int kSecLights = 5;
__host__ __device__ inline int sec_light_groups(int nl) { return (nl + kSecLights - 1) / kSecLights; }
template <int TS>
__device__ __forceinline__ void edge_secondary_body(const Scene &S, uint64_t seed, int spp, long long s0, long long n,
        const float *__restrict__ dLdI, const HitRec *__restrict__ hits, uint32_t *__restrict__ out,
        uint32_t *__restrict__ out_n, unsigned long long *ctr, int bx, int by) {
    static_assert(TS % 256 == 0 && TS <= 65536, "a tile is whole blocks of 256 samples");
    __shared__ Light Ls[kMaxLights];
    __shared__ uint32_t ql[TS * kSecLights];   // proposals that need rays: tile index | light << 16
    __shared__ int q_n;
    for (int k = threadIdx.x; k < S.nl; k += blockDim.x) {
        const float *g = S.lgeom + 12 * k;
        Light L;
        L.c = mk(g[0], g[1], g[2]); L.e1 = mk(g[3], g[4], g[5]); L.e2 = mk(g[6], g[7], g[8]);
        L.n = mk(g[9], g[10], g[11]);
        Ls[k] = L;
    }
    if (threadIdx.x == 0) q_n = 0;
    __syncthreads();
    const float geoR = *S.geo_R;
    const long long base = (long long)bx * TS;
    const int lane = threadIdx.x & 63;
    const int jbeg = by * kSecLights, jend = min(S.nl, jbeg + kSecLights);
    uint32_t n_sec = 0;
    Work wk;
    for (int k = 0; k < TS; k += 256) {
        const int li = k + (int)threadIdx.x;
        const long long i = base + li;
        v3 o, d; float w[3]; Hit h; SurfDec sd; uint32_t s; bool live = false;
        if (i < n) sec_setup(S, seed, spp, s0, i, dLdI, hits, o, d, w, h, sd, s, live);
        for (int j = jbeg; j < jend; ++j) {
            bool need = false, vp = false;
            if (live)
                need = secondary_edge<kSecPropose>(S, Ls[j], j, seed, s, nullptr, o, d, h, sd, w, nullptr, vp, n_sec,
                                                   wk, geoR);
            const unsigned long long m = __ballot(need);
            int wbase = 0;
            if (lane == 0 && m) wbase = atomicAdd(&q_n, __popcll(m));
            wbase = __shfl(wbase, 0);
            if (need) ql[wbase + lanes_below(m)] = (uint32_t)li | ((uint32_t)j << 16);
        }
    }
    __syncthreads();
    // each listed proposal's two side rays, rebuilt from its sample and
    // light exactly as the proposal built them, traced in one walk
    const int nq = q_n;
    for (int e = threadIdx.x; e - lane < nq; e += 256) {
        bool val = false, vq = false;
        long long i2 = 0;
        uint32_t j2 = 0;
        if (e < nq) {
            const uint32_t q = ql[e];
            i2 = base + (long long)(q & 0xffffu);
            j2 = q >> 16;
            v3 o, d; float w[3]; Hit h; SurfDec sd; uint32_t s; bool live;
            sec_setup(S, seed, spp, s0, i2, dLdI, hits, o, d, w, h, sd, s, live);
            v3 sides[2];
            bool vdummy = false;
            if (live && secondary_edge<kSecPropose>(S, Ls[j2], (int)j2, seed, s, nullptr, o, d, h, sd, w, nullptr,
                                                    vdummy, n_sec, wk, geoR, sides)) {
                bool bp, bm;
                n_sec += 2;
                trace_any2(S, sd.p, sides[0], sides[1], h.tri, bp, bm, wk);
                vq = !bp;
                val = bp != bm;
            }
        }
        const unsigned long long mv = __ballot(val);
        uint32_t obase = 0;
        if (lane == 0 && mv) obase = atomicAdd(out_n, (uint32_t)__popcll(mv));
        obase = (uint32_t)__shfl((int)obase, 0);
        if (val) out[obase + lanes_below(mv)] = (uint32_t)i2 | (j2 << 24) | (vq ? 1u << 30 : 0u);
    }
    flush_count(ctr, 3, n_sec);
    flush_work(ctr, wk);
}
__global__ __launch_bounds__(256) void k_edge_secondary(Scene S, uint64_t seed, int spp, long long s0, long long n,
        const float *__restrict__ dLdI, const HitRec *__restrict__ hits, uint32_t *__restrict__ out,
        uint32_t *__restrict__ out_n, unsigned long long *ctr) {
    edge_secondary_body<kSecTile>(S, seed, spp, s0, n, dLdI, hits, out, out_n, ctr, blockIdx.x, blockIdx.y);
}

// gx blocks stride over the list
__device__ __forceinline__ void edge_secondary_value_body(const Scene &S, uint64_t seed, int spp, long long s0,
        const float *__restrict__ dLdI, const HitRec *__restrict__ hits, const uint32_t *__restrict__ list,
        const uint32_t *__restrict__ list_n, double *d_pos, int bx, int gx) {
    extern __shared__ float dyn[];
    __shared__ Light Ls[kMaxLights];
    float *spec_lds = dyn;
    stage_tables(S, Ls, spec_lds);
    __syncthreads();
    const uint32_t cnt = *list_n;
    const float geoR = *S.geo_R;
    uint32_t n_dummy = 0;
    Work wk;
    for (uint32_t k = bx * blockDim.x + threadIdx.x; k < cnt; k += gx * blockDim.x) {
        uint32_t q = list[k];
        long long i = q & 0xffffffu;
        int j = (q >> 24) & 63;
        bool vp = (q >> 30) & 1u;
        v3 o, d; float w[3]; Hit h; SurfDec sd; uint32_t s; bool live;
        sec_setup(S, seed, spp, s0, i, dLdI, hits, o, d, w, h, sd, s, live);
        secondary_edge<kSecValue>(S, Ls[j], j, seed, s, spec_lds, o, d, h, sd, w, d_pos, vp, n_dummy, wk, geoR);
    }
}
__global__ __launch_bounds__(256) void k_edge_secondary_value(Scene S, uint64_t seed, int spp, long long s0,
        const float *__restrict__ dLdI, const HitRec *__restrict__ hits, const uint32_t *__restrict__ list,
        const uint32_t *__restrict__ list_n, double *d_pos) {
    edge_secondary_value_body(S, seed, spp, s0, dLdI, hits, list, list_n, d_pos, blockIdx.x, gridDim.x);
}

// ---------------------------------------------- camera silhouettes -----
// M = W*H edge samples, in three passes so that the 40 shadow rays of a
// sample run on separate lanes:
//   setup                 pick the edge, the point q on its projection, the
//                         two sides q +- offset; find the sides' camera-ray
//                         hits (k_pe_* in the single context, a walk per
//                         sample in the batched path);
//   k_pv_propose, k_pv_trace  per light, the sides whose light sample is
//                         above their horizon, queued, then one shadow ray
//                         per queued side and its visibility bit;
//   k_edge_primary_shade  one lane per side: fp64 radiance of its visible
//                         lights;
//   k_edge_primary_scatter one lane per sample: (f+ - f-) times the boundary
//                         Jacobian into the edge's two endpoints.
struct PeSample { int e, i, pix; float qx, qy; };

// The sample's edge (CDF pick), its point q on the edge's projection and the
// two side points q +- offset along the projected edge's normal, in pixels;
// false (ps.e = -1) when the sample has none.
__device__ __forceinline__ bool pe_pick(const Scene &S, uint64_t seed, int m, PeSample &ps, float &px0, float &py0,
                                        float &px1, float &py1) {
    ps.e = -1; ps.i = 0; ps.pix = -1; ps.qx = ps.qy = 0.0f;
    const int n = S.pe_n[0];
    const uint64_t Q = S.pe_Q[0];
    if (n <= 0 || Q == 0) return false;
    u4 wd = philox(seed, (uint32_t)m, 0, 2, 0);
    uint64_t target = __umul64hi(((uint64_t)wd.y << 32) | wd.x, Q);
    int i = cdf_pick_guided(S.pe_prefix, S.pe_guide, n, Q, target);
    int e = S.pe_edge[i];
    const int *ed = S.edges + 4 * e;
    float tu = u01(wd.z);
    v3 a = vpos(S, ed[0]), b = vpos(S, ed[1]);
    float ax, ay, bx, by;
    if (!project(S, a, ax, ay) || !project(S, b, bx, by)) return false;
    float qx = ax + tu * (bx - ax), qy = ay + tu * (by - ay);
    float fpx = floorf(qx), fpy = floorf(qy);
    if (!(fpx >= 0.0f && fpx < (float)S.W && fpy >= 0.0f && fpy < (float)S.H)) return false;
    v3 cam = mk(S.cam_x, S.cam_y, S.cam_z);
    v3 mv = cross(a - cam, b - cam);
    float gx = mv.x, gy = -mv.y;
    float gl = sqrtf(gx * gx + gy * gy);
    if (gl == 0.0f) return false;
    float nx = gx / gl, ny = gy / gl;
    px0 = qx + kEdgeOffPx * nx; py0 = qy + kEdgeOffPx * ny;
    px1 = qx + -1.0f * (kEdgeOffPx * nx); py1 = qy + -1.0f * (kEdgeOffPx * ny);
    ps.e = e; ps.i = i; ps.pix = (int)fpy * S.W + (int)fpx; ps.qx = qx; ps.qy = qy;
    return true;
}

// Samples in screen order.  The samples pick their edges at random, so sides
// adjacent in sample order lie far apart on the face and their shadow rays
// walk unrelated parts of the tree.  A counting sort of the samples by screen
// tile (kPvSortPx^2 pixels; the tile of the pixel of q) gives k_pv_propose an
// order in which the queued rays of a wave start close together; the
// visibility bits do not depend on it.  Each tile has kPvSortCopies
// counters, sample m counting on copy (m / 64) mod kPvSortCopies: device
// atomics on one word serialise, and the silhouette tiles are few.  The
// sort's counters (pv_aux), with key = tile kPvSortCopies + copy:
//   [(nt + 1) C]  samples per key, then (k_scan_u32) offsets: entry nt C is
//                 the number of samples with an edge;
//   [(nt + 1) C]  each key's fill counter (k_pv_order);
//   [nl]          the light queues' lengths (k_pv_propose).
// The samples are counted where they are picked (k_pe_pick, the batched
// setup); k_pv_order writes each one's index at its key's next free slot.
constexpr int kPvSortPx = 8, kPvSortCopies = 8;
__host__ __device__ inline int pv_tiles_x(int W) { return (W + kPvSortPx - 1) / kPvSortPx; }
__host__ __device__ inline int pv_tiles(int W, int H) { return pv_tiles_x(W) * ((H + kPvSortPx - 1) / kPvSortPx); }
__host__ __device__ inline int pv_keys(int W, int H) { return (pv_tiles(W, H) + 1) * kPvSortCopies; }
__host__ __device__ inline int pv_aux_len(int W, int H, int nl) { return 2 * pv_keys(W, H) + nl; }
__device__ __forceinline__ int pv_key(const Scene &S, int m, int pix) {
    const int py = pix / S.W, px = pix - py * S.W;
    const int t = (py / kPvSortPx) * pv_tiles_x(S.W) + px / kPvSortPx;
    return t * kPvSortCopies + ((m >> 6) & (kPvSortCopies - 1));
}
__device__ __forceinline__ void pv_order_body(const Scene &S, int M, const PeSample *__restrict__ ps,
        uint32_t *__restrict__ aux, uint32_t *__restrict__ perm, int bx) {
    const int m = bx * 256 + threadIdx.x;
    if (m >= M || ps[m].e < 0) return;
    const int key = pv_key(S, m, ps[m].pix);
    perm[aux[key] + atomicAdd(&aux[pv_keys(S.W, S.H) + key], 1u)] = (uint32_t)m;
}
__global__ __launch_bounds__(256) void k_pv_order(Scene S, int M, const PeSample *__restrict__ ps,
        uint32_t *__restrict__ aux, uint32_t *__restrict__ perm) {
    pv_order_body(S, M, ps, aux, perm, blockIdx.x);
}

// Batched path: one lane per sample traces both sides' camera rays in one
// walk.
__device__ __forceinline__ void edge_primary_setup_body(const Scene &S, uint64_t seed, int M,
        PeSample *__restrict__ ps_out, Hit *__restrict__ hits, unsigned long long *__restrict__ pvis,
        uint32_t *__restrict__ pv_aux, unsigned long long *ctr, int bx) {
    const int m = bx * blockDim.x + threadIdx.x;
    uint32_t n_cam = 0;
    Work wk;
    if (m < M) {
        PeSample ps;
        Hit h0; h0.tri = -1; h0.t = 0.0f; h0.b1 = h0.b2 = h0.det = 0.0f;
        Hit hs[2] = {h0, h0};
        float px0, py0, px1, py1;
        if (pe_pick(S, seed, m, ps, px0, py0, px1, py1)) {
            const v3 cam = mk(S.cam_x, S.cam_y, S.cam_z);
            trace_closest2(S, cam, camera_dir(S, px0, py0), camera_dir(S, px1, py1), hs[0], hs[1], wk);
            n_cam = 2;
            atomicAdd(&pv_aux[pv_key(S, m, ps.pix)], 1u);
        }
        ps_out[m] = ps;
        hits[2 * m] = hs[0];
        hits[2 * m + 1] = hs[1];
        pvis[2 * m] = 0ull;
        pvis[2 * m + 1] = 0ull;
    }
    flush_count(ctr, 0, n_cam);
    flush_work(ctr, wk);
}

// Single context: the side rays are camera rays through arbitrary screen
// points, too few (2 W H) to keep the chip busy walking the tree.  Their
// hits are the minimum of (t, triangle id) over the triangles whose test
// accepts the ray, bit for bit the walk's hit, found through a screen grid:
//   k_pe_tri_count  one lane per triangle: the cells (kPeCell^2 pixels, with
//                   a one-pixel border around the image for side points just
//                   outside it) that its camera footprint covers;
//   k_scan_u32      cell counts -> offsets;
//   k_pe_tri_fill   each cell's triangles as 48-byte vertex records;
//   k_pe_pick       one lane per sample: edge, point, side points;
//   k_pe_resolve    one lane per side: the tests against its cell's
//                   triangles, the minimum kept as the walk keeps it.
// The records have a fixed capacity; past it the sides walk the tree.
constexpr int kPeCell = 2;
constexpr int kPeRecPerTri = 16;     // record capacity: this many per triangle, plus one per cell
__device__ __forceinline__ int pe_cell_1d(int px) { return (px >= 0 ? px / kPeCell : -1) + 1; }   // px >= -1
__device__ __forceinline__ int pe_cell(const Scene &S, float px, float py, int ncx) {
    const int ix = min(max((int)floorf(px), -1), S.W), iy = min(max((int)floorf(py), -1), S.H);
    return pe_cell_1d(iy) * ncx + pe_cell_1d(ix);
}
// cell range of a triangle's footprint; false when empty
__device__ __forceinline__ bool pe_tri_cells(const Scene &S, int f, v3 &v0, v3 &v1, v3 &v2, int &cx0, int &cx1,
                                             int &cy0, int &cy1) {
    const int *t = S.faces + 3 * f;
    v0 = vpos(S, t[0]); v1 = vpos(S, t[1]); v2 = vpos(S, t[2]);
    int x0, x1, y0, y1;
    cam_footprint(S, v0, v1, v2, 1, x0, x1, y0, y1);
    if (x0 > x1 || y0 > y1) return false;
    cx0 = pe_cell_1d(x0); cx1 = pe_cell_1d(x1); cy0 = pe_cell_1d(y0); cy1 = pe_cell_1d(y1);
    return true;
}
__global__ __launch_bounds__(256) void k_pe_tri_count(Scene S, int ncx, uint32_t *__restrict__ cell_n) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= S.F) return;
    v3 v0, v1, v2;
    int cx0, cx1, cy0, cy1;
    if (!pe_tri_cells(S, f, v0, v1, v2, cx0, cx1, cy0, cy1)) return;
    for (int cy = cy0; cy <= cy1; ++cy)
        for (int cx = cx0; cx <= cx1; ++cx) atomicAdd(&cell_n[cy * ncx + cx], 1u);
}
__global__ __launch_bounds__(256) void k_pe_tri_fill(Scene S, int ncx, const uint32_t *__restrict__ off,
        uint32_t *__restrict__ fill, float4 *__restrict__ rec, uint32_t cap) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= S.F) return;
    v3 v0, v1, v2;
    int cx0, cx1, cy0, cy1;
    if (!pe_tri_cells(S, f, v0, v1, v2, cx0, cx1, cy0, cy1)) return;
    for (int cy = cy0; cy <= cy1; ++cy)
        for (int cx = cx0; cx <= cx1; ++cx) {
            const int c = cy * ncx + cx;
            const uint32_t slot = off[c] + atomicAdd(&fill[c], 1u);
            if (slot < cap) {
                rec[3 * (size_t)slot] = make_float4(v0.x, v0.y, v0.z, v1.x);
                rec[3 * (size_t)slot + 1] = make_float4(v1.y, v1.z, v2.x, v2.y);
                rec[3 * (size_t)slot + 2] = make_float4(v2.z, __int_as_float(f), 0.0f, 0.0f);
            }
        }
}
// (a sample without an edge gets its sides' empty hits and visibility here:
// k_pe_resolve walks only the samples with one, in screen order)
__global__ __launch_bounds__(256) void k_pe_pick(Scene S, uint64_t seed, int M, PeSample *__restrict__ ps_out,
        float2 *__restrict__ q, uint32_t *__restrict__ pv_aux, Hit *__restrict__ hits,
        unsigned long long *__restrict__ pvis) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    PeSample ps;
    float px[2], py[2];
    if (pe_pick(S, seed, m, ps, px[0], py[0], px[1], py[1])) {
        q[2 * m] = make_float2(px[0], py[0]);
        q[2 * m + 1] = make_float2(px[1], py[1]);
        atomicAdd(&pv_aux[pv_key(S, m, ps.pix)], 1u);
    } else {
        Hit h; h.tri = -1; h.t = 0.0f; h.b1 = h.b2 = h.det = 0.0f;
        hits[2 * m] = h; hits[2 * m + 1] = h;
        pvis[2 * m] = 0ull; pvis[2 * m + 1] = 0ull;
    }
    ps_out[m] = ps;
}
// Lane g takes side g % 2 of the (g / 2)-th sample with an edge in screen
// order (perm, n_edge samples): neighbouring lanes then test the triangles
// of the same or neighbouring cells, so their loops run about as long.
__global__ __launch_bounds__(256) void k_pe_resolve(Scene S, int M, int ncx, int nc, const PeSample *__restrict__ ps,
        const float2 *__restrict__ q, const uint32_t *__restrict__ off, const float4 *__restrict__ rec, uint32_t cap,
        const uint32_t *__restrict__ perm, const uint32_t *__restrict__ n_edge, Hit *__restrict__ hits,
        unsigned long long *__restrict__ pvis, unsigned long long *ctr) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t n_cam = 0;
    Work wk;
    if (g < 2 * *n_edge) {
        const int side = 2 * (int)perm[g >> 1] + (int)(g & 1);
        Hit h; h.tri = -1; h.t = 0.0f; h.b1 = h.b2 = h.det = 0.0f;
        if (ps[side >> 1].e >= 0) {
            n_cam = 1;
            const float2 p = q[side];
            const v3 o = mk(S.cam_x, S.cam_y, S.cam_z), d = camera_dir(S, p.x, p.y);
            if (off[nc] > cap) {
                h = trace_closest(S, o, d, wk);   // records overflowed: walk the tree
            } else {
                h.t = INFINITY;
                const int c = pe_cell(S, p.x, p.y, ncx);
                const uint32_t end = off[c + 1];
                // four records loaded before they are tested, so that their
                // loads overlap
                for (uint32_t k = off[c]; k < end; k += 4) {
                    float4 r[4][3];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (k + u < end)
                            for (int w = 0; w < 3; ++w) r[u][w] = rec[3 * (size_t)(k + u) + w];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        if (k + u >= end) break;
                        const float4 r0 = r[u][0], r1 = r[u][1], r2 = r[u][2];
                        const int f = __float_as_int(r2.y);
                        float t, b1, b2, det;
                        ++wk.tri;
                        if (ray_tri(o, d, mk(r0.x, r0.y, r0.z), mk(r0.w, r1.x, r1.y), mk(r1.z, r1.w, r2.x), 0.0f,
                                    INFINITY, t, b1, b2, det) &&
                            (t < h.t || (t == h.t && f < h.tri))) {
                            h.tri = f; h.t = t; h.b1 = b1; h.b2 = b2; h.det = det;
                        }
                    }
                }
            }
        }
        hits[side] = h;
        pvis[side] = 0ull;
    }
    flush_count(ctr, 0, n_cam);
    flush_work(ctr, wk);
}

// screen point of side 'side' of a primary sample (same fp32 ops as setup)
__device__ __forceinline__ void pe_side_point(const Scene &S, const PeSample &ps, int side, float &px, float &py) {
    const int *ed = S.edges + 4 * ps.e;
    v3 cam = mk(S.cam_x, S.cam_y, S.cam_z);
    v3 mv = cross(vpos(S, ed[0]) - cam, vpos(S, ed[1]) - cam);
    float gx = mv.x, gy = -mv.y;
    float gl = sqrtf(gx * gx + gy * gy);
    float nx = gx / gl, ny = gy / gl;
    float sg = side == 0 ? 1.0f : -1.0f;
    px = ps.qx + sg * (kEdgeOffPx * nx);
    py = ps.qy + sg * (kEdgeOffPx * ny);
}

// the light sample of side ms = 2 m + side toward light j; false when the
// sample has no surface or the light point is below its horizon
__device__ __forceinline__ bool pe_light(const Scene &S, uint64_t seed, const PeSample *ps_in, const Hit *hits,
        const Light &L, int j, int ms, v3 &o, v3 &d, Hit &h, SurfDec &sd, v3 &y) {
    int m = ms >> 1, side = ms & 1;
    PeSample ps = ps_in[m];
    h = hits[ms];
    if (ps.e < 0 || h.tri < 0) return false;
    float px, py;
    pe_side_point(S, ps, side, px, py);
    o = mk(S.cam_x, S.cam_y, S.cam_z);
    d = camera_dir(S, px, py);
    surf_decide(S, o, h, sd);
    LightRng rng(seed, (uint32_t)m, 2, 4);
    float u, v;
    rng.get(j, u, v);
    y = light_point(L, u, v);
    return above(sd, y);
}

// The sides' shadow rays in two kernels, as the pixel samples' (most sides
// trace nothing: the side off the face has no hit, and about half of the
// rest have the light below their horizon):
//   k_pv_propose  one block per 256 sides (in screen order) for all lights:
//                 the horizon tests; the accepted sides' indices go to each
//                 light's queue;
//   k_pv_trace    one lane per queued side, its ray rebuilt as k_pv_propose
//                 built it, traced; a clear path sets the light's bit in the
//                 side's mask.
// k_edge_primary_shade: one lane per side, the fp64 radiance of its visible
// lights summed in light order (no atomics; the fp64 shading registers stay
// out of the traversal kernel).
// k_pv_propose: one block per 256 sides in screen order (position k is
// side k & 1 of sample perm[k >> 1]) for every light, each side's surface
// decided once (the decisions of pe_light); the queues hold side indices.
__device__ __forceinline__ void pv_propose_body(const Scene &S, uint64_t seed, const PeSample *__restrict__ ps_in,
        const Hit *__restrict__ hits, const uint32_t *__restrict__ perm, uint32_t *__restrict__ aux,
        uint32_t *__restrict__ queue, uint32_t qcap, unsigned long long *ctr, int bx) {
    const int nk = pv_keys(S.W, S.H);
    const long long n = 2 * (long long)aux[nk - kPvSortCopies];   // sides of the samples with an edge
    const long long k = (long long)bx * 256 + threadIdx.x;
    int ms = 0;
    bool have = false;
    SurfDec sd;
    if (k < n) {
        ms = 2 * (int)perm[k >> 1] + (int)(k & 1);
        const Hit h = hits[ms];
        if (ps_in[ms >> 1].e >= 0 && h.tri >= 0) {
            surf_decide(S, mk(S.cam_x, S.cam_y, S.cam_z), h, sd);
            have = true;
        }
    }
    LightRng rng(seed, (uint32_t)(ms >> 1), 2, 4);
    const uint32_t n_sh = propose_all_body(S, (uint32_t)ms, queue, qcap, aux + 2 * nk, [&](int j, const Light &L) {
        if (!have) return false;
        float u, v;
        rng.get(j, u, v);
        return above(sd, light_point(L, u, v));
    });
    flush_count(ctr, 2, n_sh);
}
__global__ __launch_bounds__(256) void k_pv_propose(Scene S, uint64_t seed, const PeSample *__restrict__ ps_in,
        const Hit *__restrict__ hits, const uint32_t *__restrict__ perm, uint32_t *__restrict__ aux,
        uint32_t *__restrict__ queue, uint32_t qcap, unsigned long long *ctr) {
    pv_propose_body(S, seed, ps_in, hits, perm, aux, queue, qcap, ctr, blockIdx.x);
}
__device__ __forceinline__ void pv_trace_body(const Scene &S, uint64_t seed, const PeSample *__restrict__ ps_in,
        const Hit *__restrict__ hits, const uint32_t *__restrict__ queue, uint32_t qcap,
        const uint32_t *__restrict__ cnt, unsigned long long *__restrict__ pvis, unsigned long long *ctr, int bx,
        int j) {
    __shared__ uint32_t lq[2 * kLeafList + 64];            // the wave's list of triangle tests
    const uint32_t e = bx * kTraceBlock + threadIdx.x;
    if ((uint32_t)bx * kTraceBlock >= cnt[j]) return;   // the whole block is past the queue
    Work wk;
    if (e < cnt[j]) {
        const int ms = (int)queue[(size_t)j * qcap + e];
        v3 o, d, y;
        Hit h;
        SurfDec sd;
        if (pe_light(S, seed, ps_in, hits, light_geom(S, j), j, ms, o, d, h, sd, y) &&
            !trace_any(S, sd.p, y - sd.p, h.tri, wk, lq))
            atomicOr(&pvis[ms], 1ull << j);
    }
    flush_work(ctr, wk);
}
__global__ __launch_bounds__(kTraceBlock) void k_pv_trace(Scene S, uint64_t seed, const PeSample *__restrict__ ps_in,
        const Hit *__restrict__ hits, const uint32_t *__restrict__ queue, uint32_t qcap,
        const uint32_t *__restrict__ cnt, unsigned long long *__restrict__ pvis, unsigned long long *ctr) {
    pv_trace_body(S, seed, ps_in, hits, queue, qcap, cnt, pvis, ctr, blockIdx.x, blockIdx.y);
}

__device__ __forceinline__ void edge_primary_shade_body(const Scene &S, uint64_t seed, int M,
        const PeSample *__restrict__ ps_in, const Hit *__restrict__ hits, const unsigned long long *__restrict__ pvis,
        double *__restrict__ fbuf, unsigned long long *ctr, int bx) {
    extern __shared__ float dyn[];
    __shared__ Light Ls[kMaxLights];
    float *spec_lds = dyn;
    stage_tables(S, Ls, spec_lds);
    __syncthreads();
    const int ms = bx * blockDim.x + threadIdx.x;
    Work wk;
    if (ms < 2 * M) {
        unsigned long long mask = pvis[ms];
        ER acc[3] = {(ER)0, (ER)0, (ER)0};
        if (mask) {
            v3 o, d, y; Hit h; SurfDec sd;
            pe_light(S, seed, ps_in, hits, Ls[0], 0, ms, o, d, h, sd, y);   // o, d, h, sd
            Surf<ER> sv;
            surf_value<ER>(S, spec_lds, o, d, h, sd, sv);
            LightRng rng(seed, (uint32_t)(ms >> 1), 2, 4);
            while (mask) {
                int j = __ffsll((long long)mask) - 1;
                mask &= mask - 1;
                float u, v;
                rng.get(j, u, v);
                const Light &L = Ls[j];
                v3 yj = light_point(L, u, v);
                ER c[3];
                shade_light<ER>(sv, L, cvt<ER>(yj), light_branch(sd, L.n, yj), nullptr, c, nullptr);
                ++wk.shade;
                for (int k = 0; k < 3; ++k) acc[k] += c[k];
            }
        }
        for (int k = 0; k < 3; ++k) fbuf[3 * ms + k] = (double)acc[k];
    }
    flush_work(ctr, wk);
}
__global__ __launch_bounds__(256) void k_edge_primary_shade(Scene S, uint64_t seed, int M,
        const PeSample *__restrict__ ps_in, const Hit *__restrict__ hits, const unsigned long long *__restrict__ pvis,
        double *__restrict__ fbuf, unsigned long long *ctr) {
    edge_primary_shade_body(S, seed, M, ps_in, hits, pvis, fbuf, ctr, blockIdx.x);
}

__device__ __forceinline__ void edge_primary_scatter_body(const Scene &S, int M, const float *__restrict__ dLdI,
        const PeSample *__restrict__ ps_in, const double *__restrict__ fbuf, double *d_pos, int bx) {
    int m = bx * blockDim.x + threadIdx.x;
    if (m < M) do {
        PeSample ps = ps_in[m];
        if (ps.e < 0) break;
        const float *Gp = dLdI + 3 * ps.pix;
        const double *f = fbuf + 6 * m;
        ER df = (ER)Gp[0] * (ER)(f[0] - f[3]) + (ER)Gp[1] * (ER)(f[1] - f[4]) + (ER)Gp[2] * (ER)(f[2] - f[5]);
        if (df == (ER)0) break;
        const int *ed = S.edges + 4 * ps.e;
        ER pxs = S.ps;
        e3 C = vk<ER>(S.cam_x, S.cam_y, S.cam_z), A = cvt<ER>(vpos(S, ed[0])), B = cvt<ER>(vpos(S, ed[1]));
        e3 dq = vk<ER>(((ER)ps.qx - (ER)0.5 * (ER)S.W) * pxs, ((ER)0.5 * (ER)S.H - (ER)ps.qy) * pxs, (ER)-1);
        e3 ra = A - C, rb = B - C;
        e3 md = cross(ra, rb);
        ER gradn = pxs * sqrt(md.x * md.x + md.y * md.y);
        ER hW = (ER)0.5 * (ER)S.W, hH = (ER)0.5 * (ER)S.H;
        ER pax = hW + (ra.x / -ra.z) / pxs, pay = hH - (ra.y / -ra.z) / pxs;
        ER pbx = hW + (rb.x / -rb.z) / pxs, pby = hH - (rb.y / -rb.z) / pxs;
        ER ln = sqrt((pbx - pax) * (pbx - pax) + (pby - pay) * (pby - pay));
        int n = S.pe_n[0];
        uint64_t Q = S.pe_Q[0];
        uint64_t qe = (ps.i + 1 < n ? S.pe_prefix[ps.i + 1] : Q) - S.pe_prefix[ps.i];
        ER pe = (ER)((double)qe / (double)Q);
        ER W = df * ln / (pe * gradn * (ER)M);
        atomic_v(d_pos, S.V, ed[0], cross(rb, dq) * W);
        atomic_v(d_pos, S.V, ed[1], cross(dq, ra) * W);
    } while (0);
}
__global__ __launch_bounds__(256) void k_edge_primary_scatter(Scene S, int M, const float *__restrict__ dLdI,
        const PeSample *__restrict__ ps_in, const double *__restrict__ fbuf, double *d_pos) {
    edge_primary_scatter_body(S, M, dLdI, ps_in, fbuf, d_pos, blockIdx.x);
}

// ------------------------------------------------------- reductions ----
// gN_k = d n_k / d N_k applied to the vertex-normal adjoint
__device__ __forceinline__ void normal_adj_body(int V, const float *__restrict__ nrm, const float *__restrict__ nlen,
        const double *__restrict__ d_nrm, double *__restrict__ gN, int bx) {
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= V) return;
    double r[3] = {0.0, 0.0, 0.0};
    if (nlen[i] > 0.0f) {
        double n[3] = {nrm[i], nrm[V + i], nrm[2 * V + i]};
        double g[3] = {d_nrm[i], d_nrm[V + i], d_nrm[2 * V + i]};
        double ng = n[0] * g[0] + n[1] * g[1] + n[2] * g[2];
        for (int c = 0; c < 3; ++c) r[c] = (g[c] - n[c] * ng) / (double)nlen[i];
    }
    gN[i] = r[0]; gN[V + i] = r[1]; gN[2 * V + i] = r[2];
}
__global__ __launch_bounds__(256) void k_normal_adj(int V, const float *__restrict__ nrm, const float *__restrict__ nlen,
        const double *__restrict__ d_nrm, double *__restrict__ gN) {
    normal_adj_body(V, nrm, nlen, d_nrm, gN, blockIdx.x);
}

// d_vertices = d_pos + sum over incident faces of the cross-product adjoint
// of N_f = (v1 - v0) x (v2 - v0) with gN_f = gN_i0 + gN_i1 + gN_i2;
// also gm = R^T d_vertices for the blend transposes.
__device__ __forceinline__ void chain_gather_body(int V, const int *__restrict__ faces,
        const int *__restrict__ vf_off, const int *__restrict__ vf_idx, const float *__restrict__ pos,
        const double *__restrict__ gN, const double *__restrict__ d_pos, const PoseArgs &P,
        float *__restrict__ d_vert, float *__restrict__ gm, int bx) {
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= V) return;
    double acc[3] = {d_pos[i], d_pos[V + i], d_pos[2 * V + i]};
    for (int q = vf_off[i]; q < vf_off[i + 1]; ++q) {
        const int *t = faces + 3 * vf_idx[q];
        double g[3] = {0.0, 0.0, 0.0}, a[3], b[3];
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 3; ++c) g[c] += gN[(size_t)c * V + t[k]];
        for (int c = 0; c < 3; ++c) {
            double x0 = pos[(size_t)c * V + t[0]];
            a[c] = (double)pos[(size_t)c * V + t[1]] - x0;
            b[c] = (double)pos[(size_t)c * V + t[2]] - x0;
        }
        double ga[3] = {b[1] * g[2] - b[2] * g[1], b[2] * g[0] - b[0] * g[2], b[0] * g[1] - b[1] * g[0]};
        double gb[3] = {g[1] * a[2] - g[2] * a[1], g[2] * a[0] - g[0] * a[2], g[0] * a[1] - g[1] * a[0]};
        for (int c = 0; c < 3; ++c) {
            if (t[1] == i) acc[c] += ga[c];
            else if (t[2] == i) acc[c] += gb[c];
            else acc[c] -= ga[c] + gb[c];
        }
    }
    d_vert[i] = (float)acc[0]; d_vert[V + i] = (float)acc[1]; d_vert[2 * V + i] = (float)acc[2];
    for (int c = 0; c < 3; ++c)
        gm[(size_t)c * V + i] = (float)((P.R[c] * acc[0] + P.R[3 + c] * acc[1]) + P.R[6 + c] * acc[2]);
}
__global__ __launch_bounds__(256) void k_chain_gather(int V, const int *__restrict__ faces,
        const int *__restrict__ vf_off, const int *__restrict__ vf_idx, const float *__restrict__ pos,
        const double *__restrict__ gN, const double *__restrict__ d_pos, PoseArgs P,
        float *__restrict__ d_vert, float *__restrict__ gm) {
    chain_gather_body(V, faces, vf_off, vf_idx, pos, gN, d_pos, P, d_vert, gm, blockIdx.x);
}

// rows: [0, n_id) B_id . gm; [n_id, +n_exp) B_exp . gm; [.., +n_alb) B_alb . d_alb;
// then 9 rows dR[a][b] = sum d_v[a] vmodel[b] and 3 rows dt[a] = sum d_v[a].
// Grid (rows, chunks); each block writes one partial.
template <int BS>
__device__ __forceinline__ void param_partial_body(int V, int n_id, int n_exp, int n_alb, int chunk,
        const float *__restrict__ b_id, const float *__restrict__ b_exp, const float *__restrict__ b_alb,
        const float *__restrict__ gm, const double *__restrict__ d_alb, const float *__restrict__ d_vert,
        const float *__restrict__ vmodel, double *__restrict__ partial, int row, int ch, int nchunks) {
    size_t L = (size_t)3 * V;
    const float *x, *y = nullptr;
    const double *yd = nullptr;
    size_t n = L;
    int kb = n_id + n_exp + n_alb;
    if (row < n_id) { x = b_id + (size_t)row * L; y = gm; }
    else if (row < n_id + n_exp) { x = b_exp + (size_t)(row - n_id) * L; y = gm; }
    else if (row < kb) { x = b_alb + (size_t)(row - n_id - n_exp) * L; yd = d_alb; }
    else if (row < kb + 9) { int a = (row - kb) / 3, b = (row - kb) % 3; x = d_vert + (size_t)a * V; y = vmodel + (size_t)b * V; n = V; }
    else { x = d_vert + (size_t)(row - kb - 9) * V; n = V; }
    size_t lo = (size_t)ch * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double acc = 0.0;
    for (size_t e = lo + threadIdx.x; e < hi; e += BS)
        acc += (double)x[e] * (y ? (double)y[e] : (yd ? yd[e] : 1.0));
    __shared__ double sh[BS];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)row * nchunks + ch] = sh[0];
}
template <int BS>
__global__ __launch_bounds__(BS) void k_param_partial(int V, int n_id, int n_exp, int n_alb, int chunk,
        const float *__restrict__ b_id, const float *__restrict__ b_exp, const float *__restrict__ b_alb,
        const float *__restrict__ gm, const double *__restrict__ d_alb, const float *__restrict__ d_vert,
        const float *__restrict__ vmodel, double *__restrict__ partial) {
    param_partial_body<BS>(V, n_id, n_exp, n_alb, chunk, b_id, b_exp, b_alb, gm, d_alb, d_vert, vmodel, partial,
                           blockIdx.x, blockIdx.y, gridDim.y);
}

struct DRotArgs { double dR[27]; };   // dR/drx, dR/dry, dR/drz, row-major

__device__ __forceinline__ void param_final_body(int n_id, int n_exp, int n_alb, int nchunks,
        const double *__restrict__ partial, const DRotArgs &D, float *d_alpha, float *d_beta, float *d_delta,
        float *d_pose, int bx) {
    int row = bx * blockDim.x + threadIdx.x;
    int kb = n_id + n_exp + n_alb;
    if (row < kb) {
        double s = 0.0;
        for (int c = 0; c < nchunks; ++c) s += partial[(size_t)row * nchunks + c];
        if (row < n_id) { if (d_alpha) d_alpha[row] = (float)s; }
        else if (row < n_id + n_exp) { if (d_beta) d_beta[row - n_id] = (float)s; }
        else if (d_delta) d_delta[row - n_id - n_exp] = (float)s;
    } else if (row == kb && d_pose) {
        double dR[9], dt[3];
        // rows 9/12 use chunks over V; the V-length rows still have nchunks partials (zeros beyond V)
        for (int r = 0; r < 12; ++r) {
            double s = 0.0;
            for (int c = 0; c < nchunks; ++c) s += partial[(size_t)(kb + r) * nchunks + c];
            if (r < 9) dR[r] = s; else dt[r - 9] = s;
        }
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int r = 0; r < 9; ++r) s += dR[r] * D.dR[9 * a + r];
            d_pose[a] = (float)s;
        }
        for (int a = 0; a < 3; ++a) d_pose[3 + a] = (float)dt[a];
    }
}
__global__ void k_param_final(int n_id, int n_exp, int n_alb, int nchunks, const double *__restrict__ partial,
        DRotArgs D, float *d_alpha, float *d_beta, float *d_delta, float *d_pose) {
    param_final_body(n_id, n_exp, n_alb, nchunks, partial, D, d_alpha, d_beta, d_delta, d_pose, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_zero(float *a, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0f;
}
__global__ void k_zero_u32(unsigned int *a, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0u;
}
__global__ void k_zero_u64(unsigned long long *a, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0ull;
}
// the counters of kernels [k0, k1) (every copy)
__global__ void k_zero_ctr(unsigned long long *ctr, int k0, int k1) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 8 * kCtrSpread * (k1 - k0)) ctr[(8 * kCtrSpread * k0 + e) * kCtrPad] = 0ull;
}
__global__ __launch_bounds__(256) void k_copy(const float *__restrict__ a, float *__restrict__ b, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}
// the adjoint's accumulators and its kernels' counters cleared in one launch
// (counter words first .. first + n - 1, kCtrPad apart)
__global__ __launch_bounds__(256) void k_zero_bwd(GradBufs G, int nl3, int rr, int V3, unsigned long long *ctr,
                                                  int ctr_first, int ctr_n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < nl3) G.d_light[i] = 0.0;
    if (i < rr) G.d_spec[i] = 0.0;
    if (i < V3) { G.d_pos[i] = 0.0; G.d_nrm[i] = 0.0; G.d_alb[i] = 0.0; }
    if (i < ctr_n) ctr[(ctr_first + i) * kCtrPad] = 0ull;
}
// the requested gradients rounded to the caller's float arrays in one launch
__global__ __launch_bounds__(256) void k_grads_out(GradBufs G, const float *__restrict__ g_vert, int nl3, int rr, int V3,
        float *d_lights, float *d_spec, float *d_vertices, float *d_albedo) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (d_lights && i < nl3) d_lights[i] = (float)G.d_light[i];
    if (d_spec && i < rr) d_spec[i] = (float)G.d_spec[i];
    if (d_vertices && i < V3) d_vertices[i] = g_vert[i];
    if (d_albedo && i < V3) d_albedo[i] = (float)G.d_alb[i];
}

template <int BS>
__global__ __launch_bounds__(BS) void k_loss_partial(size_t n, const float *__restrict__ img, const float *__restrict__ tgt,
        float *__restrict__ dL, double *__restrict__ partial) {
    size_t i = (size_t)blockIdx.x * BS + threadIdx.x;
    double acc = 0.0;
    if (i < n) {
        float r = img[i] - tgt[i];
        if (dL) dL[i] = 2.0f * r;
        acc = (double)r * (double)r;
    }
    __shared__ double sh[BS];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}
template <int BS>
__global__ __launch_bounds__(BS) void k_loss_final(int nb, const double *__restrict__ partial, float *loss) {
    __shared__ double sh[BS];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += BS) acc += partial[b];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)sh[0];
}

// ====================================================================== //
//                               host side                                //
// ====================================================================== //

// Camera samples per chunk of the forward wavefront (24 B of records each).
// A render that fits in one chunk leaves its records for the adjoint; a
// larger one (very high spp) has them recomputed chunk by chunk.
// -------------------------------------------------- auxiliary buffers --
// Per pixel, the mean over its samples of the first hit's albedo (RGB, the
// interpolated vertex albedo), unit shading normal (turned toward the
// camera) and distance from the camera; a miss contributes zeros.  One lane
// per pixel, reading the render's hit records (its samples are adjacent).
__global__ __launch_bounds__(256) void k_aov(Scene S, uint64_t seed, int spp, const HitRec *__restrict__ hits,
                                            float *__restrict__ out) {
    int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix >= S.W * S.H) return;
    const v3 cam = mk(S.cam_x, S.cam_y, S.cam_z);
    float acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < spp; ++k) {
        uint32_t s = (uint32_t)((size_t)pix * spp + k);
        HitRec rec = hits[s];
        if (rec.tri < 0) continue;
        Hit h = hit_of(rec);
        int px;
        v3 d = camera_sample(S, seed, s, spp, px);
        SurfDec sd;
        surf_decide(S, cam, h, sd);
        // the value path's surface: barycentrics re-solved in fp64, as the
        // shading uses them
        Surf<float> sv;
        surf_value<float>(S, S.spec, cam, d, h, sd, sv);
        for (int c = 0; c < 3; ++c) acc[c] += sv.A[c];
        acc[3] += sv.ns.x; acc[4] += sv.ns.y; acc[5] += sv.ns.z;
        acc[6] += sv.olen;
    }
    float inv = 1.0f / (float)spp;
    for (int c = 0; c < 7; ++c) out[(size_t)pix * 7 + c] = acc[c] * inv;
}

// ------------------------------------------------------------ fitting --
// Light regulariser of the objective (Eq. 1): E_light = sum_j |l_j - m_j|^2
// with m_j the mean of light j's three channels, times w2.  Its gradient
// 2 w2 (l_j - m_j) holds whether m_j is treated as a constant or not, since
// the deviations of one light sum to zero.  One block, one lane per light.
__global__ __launch_bounds__(64) void k_light_reg(int nl, const float *__restrict__ lights, float w2,
                                                  float *__restrict__ grad, float *__restrict__ loss) {
    double e = 0.0;
    for (int j = threadIdx.x; j < nl; j += 64) {
        float r = lights[3 * j], g = lights[3 * j + 1], b = lights[3 * j + 2];
        float m = ((r + g) + b) / 3.0f;
        float d[3] = {r - m, g - m, b - m};
        for (int c = 0; c < 3; ++c) {
            e += (double)d[c] * (double)d[c];
            if (grad) grad[3 * j + c] += 2.0f * w2 * d[c];
        }
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if (threadIdx.x == 0 && loss) *loss = (float)((double)w2 * e);
}

// Adam (Kingma and Ba 2015), one thread per element:
//   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
//   p <- p - lr (m / c1) / (sqrt(v / c2) + eps),  c1 = 1 - b1^t, c2 = 1 - b2^t
// (c1, c2 computed on the host in double and rounded to float).
__global__ __launch_bounds__(256) void k_adam(int n, float *__restrict__ p, const float *__restrict__ g,
        float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2, float c1, float c2, float eps) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static constexpr long long kChunkMax = FR_CHUNK_MAX;
// shadow-boundary samples are listed per sub-range of a chunk (list size
// bounded by kSecSub * lights entries)
static constexpr long long kSecSub = 1ll << 21;
enum { kKernCamera, kKernShadow, kKernShade, kKernAdj, kKernPrimary, kKernSecondary, kNumKern };
static constexpr int kNumEvents = 8 + 2 * kNumKern;

struct fr_ctx {
    std::string err;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;           // the camera-silhouette term's stream (fr_backward)
    hipStream_t side2 = nullptr;          // the shadow-boundary term's stream (fr_backward)
    hipEvent_t fork2_ev = nullptr, join2_ev = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    uint32_t flags = 0, terms = FR_TERM_INTERIOR | FR_TERM_PRIMARY | FR_TERM_SECONDARY;
    int device = 0;
    // host-pointer mode (no FR_DEVICE_PTRS): device copies of a call's arrays,
    // and of the last render's parameter arrays (fr_backward reads them)
    std::vector<std::pair<void *, size_t>> io_buf, par_buf;
    // sizes
    int V = 0, F = 0, E = 0, n_id = 0, n_exp = 0, n_alb = 0;
    int W = 0, H = 0, nl = 0, res = 0, n_nodes = 0;
    float cam[3] = {0, 0, 0}, ps = 0;
    // model (device)
    int *faces = nullptr, *edges = nullptr, *vf_off = nullptr, *vf_idx = nullptr;
    float *mean = nullptr, *b_id = nullptr, *b_exp = nullptr, *alb_mean = nullptr, *b_alb = nullptr, *uv = nullptr;
    float *lgeom = nullptr;
    // tree order (device)
    int *sorted_tri = nullptr, *leaf_node = nullptr, *right = nullptr, *escape = nullptr;
    SubTree *subs = nullptr; int n_subs = 0;
    LbvhBufs lb{};                 // per-evaluation build (without FR_REFIT)
    int *height = nullptr, *top = nullptr, *top_off = nullptr; int n_top = 0, top_levels = 0;
    Node *nodes = nullptr;
    float4 *tris = nullptr;
    // per evaluation (device)
    double *vm_d = nullptr;
    float *vmodel = nullptr, *pos = nullptr, *nrm = nullptr, *nlen = nullptr, *alb = nullptr;
    float *ew = nullptr;
    int *tbl_edge = nullptr, *tbl_n = nullptr; uint64_t *tbl_prefix = nullptr, *tbl_Q = nullptr;
    int *tbl_guide = nullptr;        // [1 + nl][E + 1] cut-point guides of the tables
    uint32_t *es_wmax = nullptr;     // [1 + nl] largest weight per table (bits)
    uint64_t *es_csum = nullptr;     // [1 + nl][chunks] quantised sums per chunk
    uint32_t *es_ccnt = nullptr;     // [1 + nl][chunks] positive counts per chunk
    float4 *edge_rec = nullptr;      // [E][5] edge geometry for the shadow-boundary proposals
    float4 *edge_pl = nullptr;       // [E][2] face planes for their pre-test
    float *geo_R = nullptr;          // largest |coordinate| of the posed vertices
    uint32_t *sh_queue = nullptr;    // [nl][sh_cap] queued shadow rays (sample index) per light
    size_t sh_cap = 0;               // its capacity per light (samples of one chunk); fr_render only
    uint32_t *sh_cnt = nullptr;      // [nl] queue lengths
    float2 *pe_q = nullptr;          // [2 W H] silhouette sides' screen points
    uint32_t *pe_cell_n = nullptr;   // [2 cells + 1]: triangle counts, then offsets; fill counters
    float4 *pe_rec = nullptr;        // [pe_cap][3] triangle vertex records in cell order
    uint32_t pe_cap = 0;
    float *samples = nullptr; size_t samples_cap = 0;
    HitRec *hits = nullptr; unsigned long long *vis = nullptr; size_t rec_cap = 0;
    uint32_t *sec_list = nullptr, *sec_n = nullptr; size_t sec_cap = 0;
    bool records_valid = false;   // hits/vis hold every sample of the last render
    PeSample *pe_samples = nullptr; Hit *pe_hits = nullptr; double *pe_f = nullptr;
    unsigned long long *pe_vis = nullptr;
    uint32_t *pv_queue = nullptr;    // [nl][2 W H] sides with a shadow ray toward each light
    uint32_t *pv_aux = nullptr;      // [pv_aux_len]: screen-order sort counters, queue lengths
    uint32_t *pv_perm = nullptr;     // [W H] samples in screen order
    unsigned long long *ctr = nullptr;
    // gradients scratch
    double *g_light = nullptr, *g_spec = nullptr, *g_pos = nullptr, *g_nrm = nullptr, *g_alb = nullptr;
    double *g_N = nullptr;
    float *g_vert = nullptr, *g_m = nullptr;
    double *partial = nullptr; int nchunks = 0, chunk = 0;
    double *loss_partial = nullptr; int loss_nb = 0;
    // last render
    bool have_render = false, have_backward = false;
    uint64_t gen = 0;              // renders so far (single or batched)
    fr_params last{};
    uint64_t last_seed = 0; int last_spp = 0;
    long long cam_chunk = kChunkMax, last_cam_chunk = kChunkMax;   // camera samples per chunk (set / of the last render)
    PoseArgs pose{};
    DRotArgs drot{};
    // timing
    hipEvent_t ev[kNumEvents] = {};
    float ms[5] = {0, 0, 0, 0, 0};
};

static const char *kNoCtx = "no context";

static int fail(fr_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCK(c, call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            return fail((c), e_ == hipErrorOutOfMemory ? FR_ENOMEM : FR_EDEVICE, "%s: %s (%s:%d)", \
                        #call, hipGetErrorString(e_), __FILE__, __LINE__);               \
        }                                                                                \
    } while (0)

template <class T>
static int dalloc(fr_ctx *c, T **p, size_t n) {
    if (n == 0) n = 1;
    HIPCK(c, hipMalloc((void **)p, n * sizeof(T)));
    return 0;
}
template <class T>
static int upload(fr_ctx *c, T **p, const T *h, size_t n) {
    if (dalloc(c, p, n)) return c ? FR_ENOMEM : -1;
    HIPCK(c, hipMemcpy(*p, h, n * sizeof(T), hipMemcpyHostToDevice));
    return 0;
}

static void rotation(const float pose[6], double R[9]) {
    // R = Rz(rz) Ry(ry) Rx(rx); products summed left to right
    double cx = cos((double)pose[0]), sx = sin((double)pose[0]);
    double cy = cos((double)pose[1]), sy = sin((double)pose[1]);
    double cz = cos((double)pose[2]), sz = sin((double)pose[2]);
    double Rx[9] = {1, 0, 0, 0, cx, -sx, 0, sx, cx};
    double Ry[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy};
    double Rz[9] = {cz, -sz, 0, sz, cz, 0, 0, 0, 1};
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            T[3 * i + j] = (Ry[3 * i] * Rx[j] + Ry[3 * i + 1] * Rx[3 + j]) + Ry[3 * i + 2] * Rx[6 + j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            R[3 * i + j] = (Rz[3 * i] * T[j] + Rz[3 * i + 1] * T[3 + j]) + Rz[3 * i + 2] * T[6 + j];
}

static void matmul3(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

static void drotation(const float pose[6], double out[27]) {
    double cx = cos((double)pose[0]), sx = sin((double)pose[0]);
    double cy = cos((double)pose[1]), sy = sin((double)pose[1]);
    double cz = cos((double)pose[2]), sz = sin((double)pose[2]);
    double Rx[9] = {1, 0, 0, 0, cx, -sx, 0, sx, cx}, dRx[9] = {0, 0, 0, 0, -sx, -cx, 0, cx, -sx};
    double Ry[9] = {cy, 0, sy, 0, 1, 0, -sy, 0, cy}, dRy[9] = {-sy, 0, cy, 0, 0, 0, -cy, 0, -sy};
    double Rz[9] = {cz, -sz, 0, sz, cz, 0, 0, 0, 1}, dRz[9] = {-sz, -cz, 0, cz, -sz, 0, 0, 0, 0};
    double T[9];
    matmul3(Ry, dRx, T); matmul3(Rz, T, out);
    matmul3(dRy, Rx, T); matmul3(Rz, T, out + 9);
    matmul3(Ry, Rx, T); matmul3(dRz, T, out + 18);
}

// ---- topology: edges, vertex->face lists, LBVH tree order -------------
struct HostTopo {
    std::vector<int> edges, vf_off, vf_idx, sorted_tri, leaf_node, parent, right, escape;
    std::vector<int> height, top, top_off;   // refit schedule
    std::vector<SubTree> subs;
    int n_nodes = 0;
};

static bool build_edges(int V, int F, const int *faces, std::vector<int> &out) {
    std::vector<uint64_t> he;
    he.reserve(3 * (size_t)F);
    for (int f = 0; f < F; ++f)
        for (int k = 0; k < 3; ++k) {
            uint32_t a = faces[3 * f + k], b = faces[3 * f + (k + 1) % 3];
            if (a > b) std::swap(a, b);
            (void)V;
            he.push_back(((uint64_t)a << 32) | b);
        }
    std::vector<std::pair<uint64_t, int>> key(he.size());
    for (size_t i = 0; i < he.size(); ++i) key[i] = {he[i], (int)(i / 3)};
    std::sort(key.begin(), key.end());
    out.clear();
    for (size_t i = 0; i < key.size();) {
        size_t j = i + 1;
        while (j < key.size() && key[j].first == key[i].first) ++j;
        if (j - i > 2) return false;
        out.push_back((int)(key[i].first >> 32));
        out.push_back((int)(key[i].first & 0xffffffffu));
        out.push_back(key[i].second);
        out.push_back(j - i == 2 ? key[i + 1].second : -1);
        i = j;
    }
    return true;
}

static float box_area(const float *b) {
    float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx < 0 ? 0.0f : 2.0f * (dx * dy + dy * dz + dz * dx);
}
static void box_grow(float *b, const float *t) {
    for (int a = 0; a < 3; ++a) { b[a] = std::min(b[a], t[a]); b[3 + a] = std::max(b[3 + a], t[3 + a]); }
}

// Binned SAH split of perm[lo, hi), laid out depth first: a node at index
// idx covering n triangles is followed by its left subtree; its right child
// starts after the left subtree's 2 n_left - 1 nodes; its escape link points
// past its own subtree.  Leaves hold one triangle (leaf order = perm order).
static void sah_rec(const std::vector<float> &bb, const std::vector<float> &cen, std::vector<int> &perm,
                    int lo, int hi, int idx, int par, HostTopo &T) {
    const int kBins = 32;
    T.parent[idx] = par;
    int count = hi - lo;
    T.escape[idx] = idx + 2 * count - 1;
    if (count == 1) {
        T.leaf_node[lo] = idx;
        T.right[idx] = -1;
        return;
    }
    float cmin[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = lo; i < hi; ++i)
        for (int a = 0; a < 3; ++a) {
            cmin[a] = std::min(cmin[a], cen[3 * perm[i] + a]);
            cmax[a] = std::max(cmax[a], cen[3 * perm[i] + a]);
        }
    float best = INFINITY;
    int best_axis = -1, best_bin = 0;
    for (int a = 0; a < 3; ++a) {
        float ext = cmax[a] - cmin[a];
        if (!(ext > 0.0f)) continue;
        float bbox[kBins][6];
        int bcnt[kBins] = {0};
        for (int k = 0; k < kBins; ++k) {
            bbox[k][0] = bbox[k][1] = bbox[k][2] = INFINITY;
            bbox[k][3] = bbox[k][4] = bbox[k][5] = -INFINITY;
        }
        for (int i = lo; i < hi; ++i) {
            int f = perm[i];
            int k = std::min(kBins - 1, (int)((cen[3 * f + a] - cmin[a]) / ext * kBins));
            bcnt[k]++;
            box_grow(bbox[k], &bb[6 * f]);
        }
        float rarea[kBins];
        int rcnt[kBins];
        float acc[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        int n = 0;
        for (int k = kBins - 1; k > 0; --k) {
            box_grow(acc, bbox[k]);
            n += bcnt[k];
            rarea[k] = box_area(acc);
            rcnt[k] = n;
        }
        float lacc[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        int nl = 0;
        for (int k = 0; k < kBins - 1; ++k) {
            box_grow(lacc, bbox[k]);
            nl += bcnt[k];
            if (nl == 0 || rcnt[k + 1] == 0) continue;
            float cost = box_area(lacc) * (float)nl + rarea[k + 1] * (float)rcnt[k + 1];
            if (cost < best) { best = cost; best_axis = a; best_bin = k; }
        }
    }
    int mid = lo + count / 2;
    if (best_axis >= 0) {
        int a = best_axis;
        float ext = cmax[a] - cmin[a];
        auto it = std::stable_partition(perm.begin() + lo, perm.begin() + hi, [&](int f) {
            return std::min(kBins - 1, (int)((cen[3 * f + a] - cmin[a]) / ext * kBins)) <= best_bin;
        });
        int m = (int)(it - perm.begin());
        if (m > lo && m < hi) mid = m;
    }
    int nl = mid - lo;
    sah_rec(bb, cen, perm, lo, mid, idx + 1, idx, T);
    T.right[idx] = idx + 2 * nl;
    sah_rec(bb, cen, perm, mid, hi, idx + 2 * nl, idx, T);
}

static bool build_topology(const fr_model_desc *m, HostTopo &T) {
    int V = m->n_vertices, F = m->n_faces;
    if (!build_edges(V, F, m->faces, T.edges)) return false;
    std::vector<int> cnt(V + 1, 0);
    for (int f = 0; f < F; ++f)
        for (int k = 0; k < 3; ++k) cnt[m->faces[3 * f + k] + 1]++;
    T.vf_off.assign(V + 1, 0);
    for (int i = 0; i < V; ++i) T.vf_off[i + 1] = T.vf_off[i] + cnt[i + 1];
    T.vf_idx.assign(3 * (size_t)F, 0);
    std::vector<int> fill(T.vf_off.begin(), T.vf_off.end() - 1);
    for (int f = 0; f < F; ++f)         // ascending f per vertex
        for (int k = 0; k < 3; ++k) {
            int v = m->faces[3 * f + k];
            bool dup = false;
            for (int q = T.vf_off[v]; q < fill[v]; ++q) dup |= T.vf_idx[q] == f;
            if (!dup) T.vf_idx[fill[v]++] = f;
        }
    // Tree order: binned-SAH top-down build over the mean shape's triangle
    // boxes (once; every evaluation refits the boxes of this tree).
    std::vector<float> bb(6 * (size_t)F), cen(3 * (size_t)F);
    for (int f = 0; f < F; ++f)
        for (int a = 0; a < 3; ++a) {
            float x0 = m->mean[(size_t)a * V + m->faces[3 * f]], x1 = m->mean[(size_t)a * V + m->faces[3 * f + 1]],
                  x2 = m->mean[(size_t)a * V + m->faces[3 * f + 2]];
            bb[6 * f + a] = std::min(std::min(x0, x1), x2);
            bb[6 * f + 3 + a] = std::max(std::max(x0, x1), x2);
            cen[3 * f + a] = (x0 + x1 + x2) / 3.0f;
        }
    std::vector<int> perm(F);
    for (int f = 0; f < F; ++f) perm[f] = f;
    T.n_nodes = 2 * F - 1;
    T.parent.assign(T.n_nodes, -1); T.right.assign(T.n_nodes, -1); T.escape.assign(T.n_nodes, 0);
    T.leaf_node.assign(F, 0);
    sah_rec(bb, cen, perm, 0, F, 0, -1, T);
    T.sorted_tri = perm;
    // refit schedule: heights, leaf counts and first slots (children follow
    // their parent in depth-first order, so one backward pass suffices)
    int NN = T.n_nodes;
    std::vector<int> lcnt(NN, 1), slo(NN, 0);
    T.height.assign(NN, 0);
    for (int i = 0; i < F; ++i) slo[T.leaf_node[i]] = i;
    for (int n = NN - 1; n >= 0; --n)
        if (T.right[n] >= 0) {
            int l = n + 1, r = T.right[n];
            T.height[n] = 1 + std::max(T.height[l], T.height[r]);
            lcnt[n] = lcnt[l] + lcnt[r];
            slo[n] = slo[l];
        }
    std::vector<std::vector<int>> lv;
    for (int n = 0; n < NN; ++n) {
        int p = T.parent[n];
        if (lcnt[n] <= kRefitLeaves && (p < 0 || lcnt[p] > kRefitLeaves))
            T.subs.push_back(SubTree{n, slo[n], lcnt[n], T.height[n]});
        else if (lcnt[n] > kRefitLeaves) {
            if ((int)lv.size() <= T.height[n]) lv.resize(T.height[n] + 1);
            lv[T.height[n]].push_back(n);
        }
    }
    T.top_off.assign(1, 0);
    for (auto &l : lv) {
        if (l.empty()) continue;
        T.top.insert(T.top.end(), l.begin(), l.end());
        T.top_off.push_back((int)T.top.size());
    }
    return true;
}

static Scene make_scene(fr_ctx *c) {
    Scene S;
    S.V = c->V; S.F = c->F; S.W = c->W; S.H = c->H; S.nl = c->nl; S.res = c->res; S.n_nodes = c->n_nodes; S.E = c->E;
    S.cam_x = c->cam[0]; S.cam_y = c->cam[1]; S.cam_z = c->cam[2]; S.ps = c->ps;
    S.faces = c->faces; S.pos = c->pos; S.nrm = c->nrm; S.alb = c->alb; S.uv = c->uv;
    S.nodes = c->nodes; S.tris = c->tris; S.lgeom = c->lgeom;
    S.lrgb = c->last.lights; S.spec = c->last.spec; S.edges = c->edges;
    size_t E = (size_t)c->E;
    S.pe_edge = c->tbl_edge; S.pe_prefix = c->tbl_prefix; S.pe_n = c->tbl_n; S.pe_Q = c->tbl_Q;
    S.se_edge = c->tbl_edge + E; S.se_prefix = c->tbl_prefix + E; S.se_n = c->tbl_n + 1; S.se_Q = c->tbl_Q + 1;
    S.pe_guide = c->tbl_guide; S.se_guide = c->tbl_guide + (E + 1);
    S.edge_rec = c->edge_rec; S.edge_pl = c->edge_pl; S.geo_R = c->geo_R;
    return S;
}

static inline unsigned nblk(size_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

static void ev_record(fr_ctx *c, int i);
// visibility masks of samples [s0, s0 + n) (after camera_pass); the events
// ev0, ev1 (when >= 0) bracket the trace kernel, which holds all the
// traversal work
static void shadow_pass(fr_ctx *c, const Scene &S, uint64_t seed, long long s0, long long n, unsigned long long *ctr,
                        int ev0 = -1, int ev1 = -1, hipEvent_t tree = nullptr) {
    const uint32_t qcap = (uint32_t)c->sh_cap;   // >= n: fr_render sized it for this chunk size
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, c->stream, c->sh_cnt, c->nl);
    hipLaunchKernelGGL(k_sh_propose, dim3(nblk(n, 256)), dim3(256), 0, c->stream, S, seed, s0, n, c->hits,
                       c->sh_queue, qcap, c->sh_cnt, ctr);
    if (tree) (void)hipStreamWaitEvent(c->stream, tree, 0);   // the tree, built on the second stream
    if (ev0 >= 0) ev_record(c, ev0);
    hipLaunchKernelGGL(k_sh_trace, dim3(nblk(n, kTraceBlock), c->nl), dim3(kTraceBlock), 0, c->stream, S, seed, s0, c->hits,
                       c->sh_queue, qcap, c->sh_cnt, c->vis, ctr);
    if (ev1 >= 0) ev_record(c, ev1);
}
// camera hit records and cleared visibility masks of samples [s0, s0 + n)
static void camera_pass(fr_ctx *c, const Scene &S, uint64_t seed, int spp, long long s0, long long n,
                        unsigned long long *ctr) {
    hipLaunchKernelGGL(k_cam_init, dim3(nblk(n, 256)), dim3(256), 0, c->stream, S, seed, spp, s0, n, c->hits, c->vis);
    if (S.F > 0)
        hipLaunchKernelGGL(k_cam_raster, dim3(nblk((size_t)S.F * spp, 256)), dim3(256), 0, c->stream, S, spp, s0, n,
                           c->hits, c->vis, ctr);
    hipLaunchKernelGGL(k_cam_resolve, dim3(nblk(n, 256)), dim3(256), 0, c->stream, S, n, c->hits, c->vis, ctr);
}

// ------------------------------------------------ host-pointer mode ----
// A context created without FR_DEVICE_PTRS takes host arrays.  A call copies
// its input arrays into device buffers that the context keeps (one per
// argument position, grown as needed), runs exactly as in device mode on
// the context's stream, copies its output arrays back and waits for the
// stream.  fr_render's parameter arrays keep buffers of their own until the
// next render, since fr_backward reads the lights and texels of the last
// render.  Every call ends with the stream idle, so a buffer is never in use
// when a later call grows it.
struct HostCall {
    fr_ctx *c;
    std::vector<std::pair<void *, size_t>> &bufs;
    size_t slot = 0;
    int err = FR_OK;
    struct Back { void *host; const void *dev; size_t bytes; };
    std::vector<Back> back;
    HostCall(fr_ctx *c_, std::vector<std::pair<void *, size_t>> &b) : c(c_), bufs(b) {}
    void *buffer(size_t bytes) {
        if (err) return nullptr;
        if (slot == bufs.size()) bufs.push_back({nullptr, 0});
        auto &b = bufs[slot++];
        if (b.second < bytes) {
            if (b.first) (void)hipFree(b.first);
            b.first = nullptr; b.second = 0;
            const size_t cap = std::max(bytes, (size_t)256);
            const hipError_t e = hipMalloc(&b.first, cap);
            if (e != hipSuccess) {
                err = fail(c, e == hipErrorOutOfMemory ? FR_ENOMEM : FR_EDEVICE, "staging %zu bytes: %s", cap,
                           hipGetErrorString(e));
                return nullptr;
            }
            b.second = cap;
        }
        return b.first;
    }
    template <class T> T *in(const T *h, size_t n) {
        if (!h) return nullptr;
        T *d = (T *)buffer(n * sizeof(T));
        if (d && n) {
            const hipError_t e = hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, c->stream);
            if (e != hipSuccess) { err = fail(c, FR_EDEVICE, "staging copy: %s", hipGetErrorString(e)); return nullptr; }
        }
        return d;
    }
    template <class T> T *out(T *h, size_t n) {
        if (!h) return nullptr;
        T *d = (T *)buffer(n * sizeof(T));
        if (d) back.push_back({h, d, n * sizeof(T)});
        return d;
    }
    template <class T> T *inout(T *h, size_t n) {
        T *d = in(h, n);
        if (d) back.push_back({h, d, n * sizeof(T)});
        return d;
    }
    // after the call: its outputs back to the host (on success), stream idle
    int finish(int r) {
        if (r == FR_OK)
            for (const Back &b : back) {
                const hipError_t e = hipMemcpyAsync(b.host, b.dev, b.bytes, hipMemcpyDeviceToHost, c->stream);
                if (e != hipSuccess) { r = fail(c, FR_EDEVICE, "copy back: %s", hipGetErrorString(e)); break; }
            }
        const hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess && r == FR_OK) r = fail(c, FR_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
        return r;
    }
};
static inline bool device_ptrs(const fr_ctx *c) { return (c->flags & FR_DEVICE_PTRS) != 0; }

extern "C" {

int fr_create(const fr_model_desc *m, const fr_scene_desc *s, uint32_t flags, fr_ctx **out) {
    if (!out) return FR_EINVAL;
    *out = nullptr;
    if (!m || !s || (flags & ~(FR_TIMING | FR_REFIT | FR_DEVICE_PTRS))) return FR_EINVAL;
    if (m->n_vertices <= 0 || m->n_faces <= 0 || m->n_id < 0 || m->n_exp < 0 || m->n_alb < 0 ||
        !m->faces || !m->mean || !m->alb_mean || !m->uv || (m->n_id && !m->b_id) || (m->n_exp && !m->b_exp) ||
        (m->n_alb && !m->b_alb) || s->width <= 0 || s->height <= 0 || s->n_lights < 1 ||
        s->n_lights > kMaxLights || !s->light_geom || s->spec_res < 1 || s->spec_res > 64 ||
        !(s->pix_scale > 0.0f) || (long long)s->width * s->height > (1ll << 26))
        return FR_EINVAL;
    for (long long i = 0; i < 3ll * m->n_faces; ++i)
        if (m->faces[i] < 0 || m->faces[i] >= m->n_vertices) return FR_EINVAL;
    for (int j = 0; j < s->n_lights; ++j)
        for (int k = 0; k < 12; ++k)
            if (!std::isfinite(s->light_geom[12 * j + k])) return FR_EINVAL;
    fr_ctx *c = new fr_ctx();
    c->flags = flags;
    HostTopo T;
    if (!build_topology(m, T)) { delete c; return FR_EINVAL; }
    if (T.edges.size() / 4 > (size_t)1 << 21) { delete c; return FR_EINVAL; }   // edge-table integer range
    c->V = m->n_vertices; c->F = m->n_faces; c->E = (int)(T.edges.size() / 4);
    c->n_id = m->n_id; c->n_exp = m->n_exp; c->n_alb = m->n_alb;
    c->W = s->width; c->H = s->height; c->nl = s->n_lights; c->res = s->spec_res; c->n_nodes = T.n_nodes;
    c->n_subs = (int)T.subs.size(); c->n_top = (int)T.top.size(); c->top_levels = (int)T.top_off.size() - 1;
    for (int a = 0; a < 3; ++a) c->cam[a] = s->cam[a];
    c->ps = s->pix_scale;
    size_t V3 = 3 * (size_t)c->V;
    int rc = 0;
    auto R = [&](int r) { if (r && !rc) rc = r; return r; };
    (void)hipGetDevice(&c->device);
    if (R(upload(c, &c->faces, m->faces, 3 * (size_t)c->F)) || R(upload(c, &c->edges, T.edges.data(), T.edges.size())) ||
        R(upload(c, &c->vf_off, T.vf_off.data(), T.vf_off.size())) || R(upload(c, &c->vf_idx, T.vf_idx.data(), T.vf_idx.size())) ||
        R(upload(c, &c->mean, m->mean, V3)) || R(upload(c, &c->alb_mean, m->alb_mean, V3)) ||
        R(upload(c, &c->uv, m->uv, 2 * (size_t)c->V)) ||
        R(upload(c, &c->b_id, m->n_id ? m->b_id : m->mean, m->n_id ? c->n_id * V3 : 1)) ||
        R(upload(c, &c->b_exp, m->n_exp ? m->b_exp : m->mean, m->n_exp ? c->n_exp * V3 : 1)) ||
        R(upload(c, &c->b_alb, m->n_alb ? m->b_alb : m->mean, m->n_alb ? c->n_alb * V3 : 1)) ||
        R(upload(c, &c->lgeom, s->light_geom, 12 * (size_t)c->nl)) ||
        R(upload(c, &c->sorted_tri, T.sorted_tri.data(), T.sorted_tri.size())) ||
        R(upload(c, &c->leaf_node, T.leaf_node.data(), T.leaf_node.size())) ||
        R(upload(c, &c->right, T.right.data(), T.right.size())) ||
        R(upload(c, &c->escape, T.escape.data(), T.escape.size())) ||
        R(upload(c, &c->subs, T.subs.data(), T.subs.size())) || R(upload(c, &c->height, T.height.data(), T.height.size())) ||
        R(upload(c, &c->top, T.top.empty() ? T.height.data() : T.top.data(), std::max<size_t>(1, T.top.size()))) ||
        R(upload(c, &c->top_off, T.top_off.data(), T.top_off.size())) ||
        R(dalloc(c, &c->nodes, (size_t)c->n_nodes)) ||
        R(dalloc(c, &c->tris, 3 * (size_t)c->F)) ||
        R(dalloc(c, &c->vmodel, V3)) || R(dalloc(c, &c->vm_d, V3)) || R(dalloc(c, &c->pos, V3)) || R(dalloc(c, &c->nrm, V3)) ||
        R(dalloc(c, &c->nlen, (size_t)c->V)) || R(dalloc(c, &c->alb, V3)) ||
        R(dalloc(c, &c->ew, (size_t)(1 + c->nl) * c->E)) ||
        R(dalloc(c, &c->tbl_edge, (size_t)(1 + c->nl) * c->E)) || R(dalloc(c, &c->tbl_prefix, (size_t)(1 + c->nl) * c->E)) ||
        R(dalloc(c, &c->tbl_n, (size_t)(1 + c->nl))) || R(dalloc(c, &c->tbl_Q, (size_t)(1 + c->nl))) ||
        R(dalloc(c, &c->tbl_guide, (size_t)(1 + c->nl) * (c->E + 1))) ||
        R(dalloc(c, &c->es_wmax, (size_t)(1 + c->nl))) || R(dalloc(c, &c->sh_cnt, (size_t)c->nl)) ||
        R(dalloc(c, &c->es_csum, (size_t)(1 + c->nl) * nblk(c->E, kEsChunk))) ||
        R(dalloc(c, &c->es_ccnt, (size_t)(1 + c->nl) * nblk(c->E, kEsChunk))) || R(dalloc(c, &c->edge_rec, (size_t)5 * c->E)) ||
        R(dalloc(c, &c->edge_pl, (size_t)2 * c->E)) || R(dalloc(c, &c->geo_R, 1)) ||
        R(dalloc(c, &c->ctr, (size_t)kCtrPerKern * kNumKern)) || R(dalloc(c, &c->sec_n, 1)) ||
        R(dalloc(c, &c->pe_samples, (size_t)c->W * c->H)) || R(dalloc(c, &c->pe_hits, 2 * (size_t)c->W * c->H)) ||
        R(dalloc(c, &c->pe_f, 6 * (size_t)c->W * c->H)) || R(dalloc(c, &c->pe_vis, 2 * (size_t)c->W * c->H)) ||
        R(dalloc(c, &c->pe_q, 2 * (size_t)c->W * c->H)) ||
        R(dalloc(c, &c->pv_queue, 2 * (size_t)c->W * c->H * c->nl)) ||
        R(dalloc(c, &c->pv_aux, (size_t)pv_aux_len(c->W, c->H, c->nl))) || R(dalloc(c, &c->pv_perm, (size_t)c->W * c->H)) ||
        R(dalloc(c, &c->pe_cell_n, 2 * (size_t)(c->W / kPeCell + 2) * (c->H / kPeCell + 2) + 1)) ||
        R(dalloc(c, &c->pe_rec, 3 * ((size_t)kPeRecPerTri * c->F + (size_t)(c->W / kPeCell + 2) * (c->H / kPeCell + 2)))) ||
        R(dalloc(c, &c->g_light, 3 * (size_t)c->nl)) || R(dalloc(c, &c->g_spec, (size_t)c->res * c->res)) ||
        R(dalloc(c, &c->g_pos, V3)) || R(dalloc(c, &c->g_nrm, V3)) || R(dalloc(c, &c->g_alb, V3)) ||
        R(dalloc(c, &c->g_N, V3)) || R(dalloc(c, &c->g_vert, V3)) || R(dalloc(c, &c->g_m, V3))) {
        int code = rc ? rc : FR_ENOMEM;
        fr_destroy(c);
        return code;
    }
    if (!(flags & FR_REFIT)) {
        int F = c->F, nb = (int)nblk(F, kSortTile);
        LbvhBufs &L = c->lb;
        L.nb = nb;
        if (dalloc(c, &L.key[0], F) || dalloc(c, &L.key[1], F) || dalloc(c, &L.val[0], F) || dalloc(c, &L.val[1], F) ||
            dalloc(c, &L.hist, (size_t)256 * nb) || dalloc(c, &L.bounds, 6) || dalloc(c, &L.child, 2 * (size_t)F) ||
            dalloc(c, &L.parent, 2 * (size_t)F) || dalloc(c, &L.first, (size_t)F) || dalloc(c, &L.last, (size_t)F) ||
            dalloc(c, &L.pre, 2 * (size_t)F) || dalloc(c, &L.arrive, (size_t)F) || dalloc(c, &L.box, 12 * (size_t)F) ||
            dalloc(c, &L.roots, (size_t)F) || dalloc(c, &L.n_roots, 1) || dalloc(c, &L.top_idx, (size_t)F) ||
            dalloc(c, &L.n_top, 1) || dalloc(c, &L.top_node, (size_t)F)) {
            fr_destroy(c);
            return FR_ENOMEM;
        }
        (void)hipMemset(L.arrive, 0, sizeof(unsigned int) * F);
    }
    c->chunk = 16384;
    c->nchunks = (int)((V3 + c->chunk - 1) / c->chunk);
    int rows = c->n_id + c->n_exp + c->n_alb + 12;
    c->loss_nb = (int)nblk(V3 > (size_t)c->W * c->H * 3 ? V3 : (size_t)c->W * c->H * 3, 256);
    if (dalloc(c, &c->partial, (size_t)rows * c->nchunks) || dalloc(c, &c->loss_partial, (size_t)c->loss_nb)) {
        fr_destroy(c);
        return FR_ENOMEM;
    }
    (void)hipMemset(c->ctr, 0, (size_t)kCtrPerKern * kNumKern * sizeof(unsigned long long));
    if (flags & FR_TIMING)
        for (int i = 0; i < kNumEvents; ++i) (void)hipEventCreate(&c->ev[i]);
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork2_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join2_ev, hipEventDisableTiming) != hipSuccess) {
        fr_destroy(c);
        return FR_EDEVICE;
    }
    if (hipDeviceSynchronize() != hipSuccess) { fr_destroy(c); return FR_EDEVICE; }
    *out = c;
    return FR_OK;
}

int fr_set_stream(fr_ctx *c, void *stream) {
    if (!c) return FR_EINVAL;
    c->stream = (hipStream_t)stream;
    return FR_OK;
}

int fr_set_chunk(fr_ctx *c, int32_t samples) {
    if (!c || samples < 1 || samples > FR_CHUNK_MAX) return FR_EINVAL;
    c->cam_chunk = samples;
    return FR_OK;
}

int fr_set_terms(fr_ctx *c, uint32_t terms) {
    if (!c || (terms & ~7u)) return FR_EINVAL;
    c->terms = terms;
    return FR_OK;
}

static void lbvh_build(fr_ctx *c, hipStream_t st) {
    const int F = c->F, nb = c->lb.nb;
    LbvhBufs &L = c->lb;
    hipLaunchKernelGGL(k_lbvh_bounds_init, dim3(1), dim3(64), 0, st, L.bounds, L.n_top, L.n_roots);
    hipLaunchKernelGGL(k_lbvh_bounds, dim3(nblk(F, 256)), dim3(256), 0, st, F, c->pos, c->V, c->faces, L.bounds);
    hipLaunchKernelGGL(k_lbvh_morton, dim3(nblk(F, 256)), dim3(256), 0, st, F, c->pos, c->V, c->faces, L.bounds,
                       L.key[0], L.val[0]);
    for (int pass = 0; pass < 4; ++pass) {
        int in = pass & 1, out = in ^ 1;
        hipLaunchKernelGGL(k_sort_hist, dim3(nb), dim3(256), 0, st, F, 8 * pass, L.key[in], L.hist, nb);
        hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, 256 * nb, L.hist);
        hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(256), 0, st, F, 8 * pass, L.key[in], L.val[in], L.hist,
                           nb, L.key[out], L.val[out]);
    }
    if (F > 1)
        hipLaunchKernelGGL(k_lbvh_karras, dim3(nblk(F - 1, 256)), dim3(256), 0, st, F, L.key[0], L.child,
                           L.parent, L.first, L.last, L.top_idx, L.n_top, L.top_node);
    hipLaunchKernelGGL(k_lbvh_layout, dim3(nblk(2 * (size_t)F - 1, 256)), dim3(256), 0, st, F, L.child, L.parent,
                       L.first, L.pre);
    hipLaunchKernelGGL(k_lbvh_boxes, dim3(nblk(F, kBoxTile)), dim3(kBoxTile), 0, st, F, c->faces, c->pos, c->V,
                       L.val[0], L.child, L.parent, L.first, L.last, L.pre, L.box, c->nodes, c->tris,
                       L.roots, L.n_roots);
    if (F > 1)
        hipLaunchKernelGGL(k_lbvh_boxes_top, dim3(1), dim3(1024), 0, st, F, L.child, L.parent, L.first, L.last,
                           L.pre, L.top_idx, L.top_node, L.n_top, L.arrive, L.box, c->nodes, L.roots, L.n_roots);
}

static int blend_impl(fr_ctx *c, const float *alpha, const float *beta, const float *delta, const float *pose) {
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(pose[k])) return fail(c, FR_EINVAL, "fr_blend: non-finite pose[%d]", k);
    rotation(pose, c->pose.R);
    for (int k = 0; k < 3; ++k) c->pose.t[k] = (double)pose[3 + k];
    drotation(pose, c->drot.dR);
    hipLaunchKernelGGL(k_blend, dim3(nblk(c->V, 64), 6), dim3(64), 0, c->stream, c->V, c->n_id, c->n_exp, c->n_alb,
                       c->mean, c->b_id, c->b_exp, c->alb_mean, c->b_alb, alpha, beta, delta,
                       c->vm_d, c->vmodel, c->alb, c->geo_R);
    hipLaunchKernelGGL(k_pose, dim3(nblk(c->V, 256)), dim3(256), 0, c->stream, c->V, c->vm_d, c->pose, c->pos,
                       c->geo_R);
    hipLaunchKernelGGL(k_normals, dim3(nblk(c->V, 256)), dim3(256), 0, c->stream, c->V, c->faces, c->vf_off, c->vf_idx,
                       c->pos, c->nrm, c->nlen);
    HIPCK(c, hipGetLastError());
    return FR_OK;
}

static int blend_call(fr_ctx *c, const float *alpha, const float *beta, const float *delta,
                      const float *pose, float *out_vertices, float *out_albedo) {
    if (!c) return FR_EINVAL;
    c->err.clear();
    if ((c->n_id && !alpha) || (c->n_exp && !beta) || (c->n_alb && !delta) || !pose)
        return fail(c, FR_EINVAL, "fr_blend: null argument");
    int r = blend_impl(c, alpha, beta, delta, pose);
    if (r) return r;
    size_t V3 = 3 * (size_t)c->V;
    if (out_vertices) hipLaunchKernelGGL(k_copy, dim3(nblk(V3, 256)), dim3(256), 0, c->stream, c->pos, out_vertices, V3);
    if (out_albedo) hipLaunchKernelGGL(k_copy, dim3(nblk(V3, 256)), dim3(256), 0, c->stream, c->alb, out_albedo, V3);
    HIPCK(c, hipGetLastError());
    return FR_OK;
}

static void ev_record(fr_ctx *c, int i) {
    if (c->flags & FR_TIMING) (void)hipEventRecord(c->ev[i], c->stream);
}

static int render_call(fr_ctx *c, const fr_params *p, uint64_t seed, int32_t spp, float *out) {
    if (!c) return FR_EINVAL;
    c->err.clear();
    if (!p || !out || !p->lights || !p->spec || !p->pose || (c->n_id && !p->alpha) || (c->n_exp && !p->beta) ||
        (c->n_alb && !p->delta))
        return fail(c, FR_EINVAL, "fr_render: null argument");
    if (spp < 1 || spp > 4096) return fail(c, FR_EINVAL, "fr_render: spp %d out of [1, 4096]", spp);
    long long N = (long long)c->W * c->H * spp;
    if (N > (1ll << 31) - 1) return fail(c, FR_EINVAL, "fr_render: W*H*spp too large");
    if ((size_t)N * 3 > c->samples_cap) {
        if (c->samples) (void)hipFree(c->samples);
        c->samples = nullptr;
        c->samples_cap = 0;
        HIPCK(c, hipMalloc((void **)&c->samples, (size_t)N * 3 * sizeof(float)));
        c->samples_cap = (size_t)N * 3;
    }
    const long long kChunk = c->cam_chunk;
    size_t rec = (size_t)std::min(N, kChunk);
    if (rec > c->rec_cap) {
        if (c->hits) (void)hipFree(c->hits);
        if (c->vis) (void)hipFree(c->vis);
        c->hits = nullptr; c->vis = nullptr; c->rec_cap = 0;
        HIPCK(c, hipMalloc((void **)&c->hits, rec * sizeof(HitRec)));
        HIPCK(c, hipMalloc((void **)&c->vis, rec * sizeof(unsigned long long)));
        c->rec_cap = rec;
    }
    // the shadow-ray queue has its own capacity: the batched path enlarges
    // the hit records (rec_cap) without it
    if (rec > c->sh_cap) {
        if (c->sh_queue) (void)hipFree(c->sh_queue);
        c->sh_queue = nullptr; c->sh_cap = 0;
        HIPCK(c, hipMalloc((void **)&c->sh_queue, rec * c->nl * sizeof(uint32_t)));
        c->sh_cap = rec;
    }
    size_t sec = (size_t)std::min(N, kSecSub) * c->nl;
    if (sec > c->sec_cap) {
        if (c->sec_list) (void)hipFree(c->sec_list);
        c->sec_list = nullptr; c->sec_cap = 0;
        HIPCK(c, hipMalloc((void **)&c->sec_list, sec * sizeof(uint32_t)));
        c->sec_cap = sec;
    }
    c->have_render = false;
    c->records_valid = false;
    c->last_cam_chunk = kChunk;
    c->last = *p;
    c->last_seed = seed;
    c->last_spp = spp;
    ev_record(c, 0);
    int r = blend_impl(c, p->alpha, p->beta, p->delta, p->pose);
    if (r) return r;
    ev_record(c, 1);
    // The tree is built on the context's second stream.  Only the shadow
    // rays read it: the screen-space camera step, the shadow-ray proposals
    // and the edge tables run beside the build on the context's stream,
    // which waits for it before the first shadow-ray trace.
    (void)hipEventRecord(c->fork_ev, c->stream);
    (void)hipStreamWaitEvent(c->side, c->fork_ev, 0);
    if (!(c->flags & FR_REFIT)) {
        lbvh_build(c, c->side);
    } else {
        hipLaunchKernelGGL(k_refit_sub, dim3(c->n_subs), dim3(256), 0, c->side, c->subs, c->faces, c->pos, c->V,
                           c->sorted_tri, c->leaf_node, c->height, c->right, c->escape, c->nodes, c->tris);
        if (c->n_top > 0)
            hipLaunchKernelGGL(k_refit_top, dim3(1), dim3(256), 0, c->side, c->n_top, c->top, c->top_off,
                               c->top_levels, c->right, c->escape, c->nodes);
    }
    if (c->flags & FR_TIMING) (void)hipEventRecord(c->ev[2], c->side);
    (void)hipEventRecord(c->join_ev, c->side);
    ev_record(c, 7);
    Scene S = make_scene(c);
    hipLaunchKernelGGL(k_edge_weights, dim3(nblk(c->E, 256)), dim3(256), 0, c->stream, S, c->lgeom, c->ew, c->edge_rec,
                       c->edge_pl);
    {
        const dim3 g(nblk(c->E, kEsChunk), 1 + c->nl);
        hipLaunchKernelGGL(k_zero_u32, dim3(nblk(1 + c->nl, 64)), dim3(64), 0, c->stream, c->es_wmax, 1 + c->nl);
        hipLaunchKernelGGL(k_es_max, g, dim3(256), 0, c->stream, c->E, c->ew, c->es_wmax);
        hipLaunchKernelGGL(k_es_sum, g, dim3(256), 0, c->stream, c->E, c->ew, c->es_wmax, c->es_csum, c->es_ccnt);
        hipLaunchKernelGGL(k_es_scan, g, dim3(256), 0, c->stream, c->E, c->ew, c->es_wmax, c->es_csum, c->es_ccnt,
                           c->tbl_edge, c->tbl_prefix, c->tbl_n, c->tbl_Q);
        hipLaunchKernelGGL(k_es_guide, g, dim3(256), 0, c->stream, c->E, c->tbl_prefix, c->tbl_n, c->tbl_Q,
                           c->tbl_guide);
    }
    ev_record(c, 3);
    hipLaunchKernelGGL(k_zero_ctr, dim3(nblk(8 * kCtrSpread * kKernAdj, 256)), dim3(256), 0, c->stream, c->ctr, 0, kKernAdj);
    size_t lds = (size_t)c->res * c->res * sizeof(float);
    for (long long s0 = 0; s0 < N; s0 += kChunk) {
        long long n = std::min(kChunk, N - s0);
        ev_record(c, 8 + 2 * kKernCamera);
        camera_pass(c, S, seed, spp, s0, n, c->ctr + kCtrPerKern * kKernCamera);
        ev_record(c, 9 + 2 * kKernCamera);
        shadow_pass(c, S, seed, s0, n, c->ctr + kCtrPerKern * kKernShadow, 8 + 2 * kKernShadow, 9 + 2 * kKernShadow,
                    s0 == 0 ? c->join_ev : nullptr);
        ev_record(c, 8 + 2 * kKernShade);
        hipLaunchKernelGGL(k_fwd_shade, dim3(nblk(n, 256)), dim3(256), lds, c->stream, S, seed, spp, s0, n,
                           c->hits, c->vis, c->samples, c->ctr + kCtrPerKern * kKernShade);
        ev_record(c, 9 + 2 * kKernShade);
    }
    hipLaunchKernelGGL(k_pixel_mean, dim3(nblk((size_t)c->W * c->H, 256)), dim3(256), 0, c->stream,
                       c->W * c->H, spp, c->samples, out);
    ev_record(c, 4);
    HIPCK(c, hipGetLastError());
    c->records_valid = N <= kChunk;
    c->have_render = true;
    c->have_backward = false;
    ++c->gen;
    return FR_OK;
}

// The camera-silhouette term on stream st (every kernel of it, between the
// phase's events).
static void primary_pass(fr_ctx *c, const Scene &S, const float *dLdI, hipStream_t st) {
    if (c->flags & FR_TIMING) (void)hipEventRecord(c->ev[8 + 2 * kKernPrimary], st);
    const size_t lds1 = (size_t)c->res * c->res * sizeof(float);
    int M = c->W * c->H;
    unsigned long long *pctr = c->ctr + kCtrPerKern * kKernPrimary;
    const int ncx = c->W / kPeCell + 2, nc = ncx * (c->H / kPeCell + 2);
    const uint32_t cap = (uint32_t)((size_t)kPeRecPerTri * c->F + nc);
    hipLaunchKernelGGL(k_zero_u32, dim3(nblk(2 * (size_t)nc + 1, 256)), dim3(256), 0, st, c->pe_cell_n,
                       2 * nc + 1);
    hipLaunchKernelGGL(k_pe_tri_count, dim3(nblk(c->F, 256)), dim3(256), 0, st, S, ncx, c->pe_cell_n);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, nc + 1, c->pe_cell_n);
    hipLaunchKernelGGL(k_pe_tri_fill, dim3(nblk(c->F, 256)), dim3(256), 0, st, S, ncx, c->pe_cell_n,
                       c->pe_cell_n + nc + 1, c->pe_rec, cap);
    const int pv_n = pv_aux_len(c->W, c->H, c->nl), pv_nk = pv_keys(c->W, c->H);
    hipLaunchKernelGGL(k_zero_u32, dim3(nblk(pv_n, 256)), dim3(256), 0, st, c->pv_aux, pv_n);
    hipLaunchKernelGGL(k_pe_pick, dim3(nblk(M, 256)), dim3(256), 0, st, S, c->last_seed, M, c->pe_samples,
                       c->pe_q, c->pv_aux, c->pe_hits, c->pe_vis);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, pv_nk, c->pv_aux);
    hipLaunchKernelGGL(k_pv_order, dim3(nblk(M, 256)), dim3(256), 0, st, S, M, c->pe_samples, c->pv_aux,
                       c->pv_perm);
    hipLaunchKernelGGL(k_pe_resolve, dim3(nblk(2 * (size_t)M, 256)), dim3(256), 0, st, S, M, ncx, nc,
                       c->pe_samples, c->pe_q, c->pe_cell_n, c->pe_rec, cap, c->pv_perm,
                       c->pv_aux + pv_tiles(c->W, c->H) * kPvSortCopies, c->pe_hits, c->pe_vis, pctr);
    const uint32_t pv_cap = 2 * (uint32_t)M;
    hipLaunchKernelGGL(k_pv_propose, dim3(nblk((size_t)pv_cap, 256)), dim3(256), 0, st, S, c->last_seed, c->pe_samples,
                       c->pe_hits, c->pv_perm, c->pv_aux, c->pv_queue, pv_cap, pctr);
    hipLaunchKernelGGL(k_pv_trace, dim3(nblk((size_t)pv_cap, kTraceBlock), c->nl), dim3(kTraceBlock), 0, st, S,
                       c->last_seed, c->pe_samples, c->pe_hits, c->pv_queue, pv_cap, c->pv_aux + 2 * pv_nk,
                       c->pe_vis, pctr);
    hipLaunchKernelGGL(k_edge_primary_shade, dim3(nblk((size_t)2 * M, 256)), dim3(256), lds1, st,
                       S, c->last_seed, M, c->pe_samples, c->pe_hits, c->pe_vis, c->pe_f, pctr);
    hipLaunchKernelGGL(k_edge_primary_scatter, dim3(nblk(M, 256)), dim3(256), 0, st,
                       S, M, dLdI, c->pe_samples, c->pe_f, c->g_pos);
    if (c->flags & FR_TIMING) (void)hipEventRecord(c->ev[9 + 2 * kKernPrimary], st);
}

static int backward_call(fr_ctx *c, const float *dLdI, const fr_grads *g) {
    if (!c) return FR_EINVAL;
    c->err.clear();
    if (!c->have_render) return fail(c, FR_ESTATE, "fr_backward: no prior fr_render");
    if (!dLdI || !g) return fail(c, FR_EINVAL, "fr_backward: null argument");
    size_t V3 = 3 * (size_t)c->V;
    const int rr = c->res * c->res, nl3 = 3 * c->nl;
    ev_record(c, 5);
    GradBufs G{c->g_light, c->g_spec, c->g_pos, c->g_nrm, c->g_alb};
    hipLaunchKernelGGL(k_zero_bwd, dim3(nblk(std::max({V3, (size_t)rr, (size_t)nl3,
                                                       (size_t)8 * kCtrSpread * (kNumKern - kKernAdj)}), 256)),
                       dim3(256), 0, c->stream, G, nl3, rr, (int)V3, c->ctr, 8 * kCtrSpread * kKernAdj,
                       8 * kCtrSpread * (kNumKern - kKernAdj));
    Scene S = make_scene(c);
    long long N = (long long)c->W * c->H * c->last_spp;
    const long long kChunk = c->last_cam_chunk;
    size_t lds = ((size_t)2 * c->res * c->res + (size_t)kLightCopies * light_stride(c->nl)) * sizeof(float);
    size_t lds1 = (size_t)c->res * c->res * sizeof(float);
    // The silhouette term reads none of the other terms' scratch and adds
    // into the vertex gradient with atomics, as they do: it runs on the
    // context's second stream beside them.  Its rays are too few to fill the
    // chip, and the other terms' kernels fill what it leaves idle.
    const bool side = (c->terms & FR_TERM_PRIMARY) != 0;
    if (side) {
        (void)hipEventRecord(c->fork_ev, c->stream);
        (void)hipStreamWaitEvent(c->side, c->fork_ev, 0);
        primary_pass(c, S, dLdI, c->side);
        (void)hipEventRecord(c->join_ev, c->side);
    }
    for (long long s0 = 0; s0 < N; s0 += kChunk) {
        long long n = std::min(kChunk, N - s0);
        if (!c->records_valid) {   // recompute this chunk's hit records and visibility
            camera_pass(c, S, c->last_seed, c->last_spp, s0, n, c->ctr + kCtrPerKern * kKernAdj);
            shadow_pass(c, S, c->last_seed, s0, n, c->ctr + kCtrPerKern * kKernAdj);
        }
        // The shadow-boundary term, bound by the latency of its dependent
        // loads, runs on a third stream beside the interior adjoint, which is
        // bound by its arithmetic; both read this chunk's records and add
        // into the gradients with atomics.  The context's stream waits for
        // it before the next chunk's records replace these.
        const bool sec = (c->terms & FR_TERM_SECONDARY) != 0, third = sec && (c->terms & FR_TERM_INTERIOR);
        const hipStream_t st2 = third ? c->side2 : c->stream;
        if (third) {
            (void)hipEventRecord(c->fork2_ev, c->stream);
            (void)hipStreamWaitEvent(c->side2, c->fork2_ev, 0);
        }
        if (c->flags & FR_TIMING) (void)hipEventRecord(c->ev[8 + 2 * kKernSecondary], st2);
        if (sec)
            for (long long o = 0; o < n; o += kSecSub) {
                long long m = std::min(kSecSub, n - o);
                hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st2, c->sec_n, 1);
                hipLaunchKernelGGL(k_edge_secondary, dim3(nblk(m, kSecTile), sec_light_groups(c->nl)), dim3(256), 0, st2, S,
                                   c->last_seed, c->last_spp, s0 + o, m, dLdI, c->hits + o, c->sec_list, c->sec_n,
                                   c->ctr + kCtrPerKern * kKernSecondary);
                hipLaunchKernelGGL(k_edge_secondary_value, dim3(1024), dim3(256), lds1, st2, S, c->last_seed,
                                   c->last_spp, s0 + o, dLdI, c->hits + o, c->sec_list, c->sec_n, c->g_pos);
            }
        if (c->flags & FR_TIMING) (void)hipEventRecord(c->ev[9 + 2 * kKernSecondary], st2);
        ev_record(c, 8 + 2 * kKernAdj);
        if (c->terms & FR_TERM_INTERIOR)
            hipLaunchKernelGGL(k_render_adj, dim3(nblk(n, 256)), dim3(256), lds, c->stream, S, c->last_seed,
                               c->last_spp, s0, n, dLdI, G, c->hits, c->vis, c->ctr + kCtrPerKern * kKernAdj);
        ev_record(c, 9 + 2 * kKernAdj);
        if (third) {
            (void)hipEventRecord(c->join2_ev, c->side2);
            (void)hipStreamWaitEvent(c->stream, c->join2_ev, 0);
        }
    }
    if (side) (void)hipStreamWaitEvent(c->stream, c->join_ev, 0);
    hipLaunchKernelGGL(k_normal_adj, dim3(nblk(c->V, 256)), dim3(256), 0, c->stream, c->V, c->nrm, c->nlen, c->g_nrm, c->g_N);
    hipLaunchKernelGGL(k_chain_gather, dim3(nblk(c->V, 256)), dim3(256), 0, c->stream, c->V, c->faces, c->vf_off, c->vf_idx,
                       c->pos, c->g_N, c->g_pos, c->pose, c->g_vert, c->g_m);
    int rows = c->n_id + c->n_exp + c->n_alb + 12;
    bool want_params = g->d_alpha || g->d_beta || g->d_delta || g->d_pose;
    if (want_params) {
        hipLaunchKernelGGL(k_param_partial<256>, dim3(rows, c->nchunks), dim3(256), 0, c->stream, c->V, c->n_id, c->n_exp,
                           c->n_alb, c->chunk, c->b_id, c->b_exp, c->b_alb, c->g_m, c->g_alb, c->g_vert, c->vmodel, c->partial);
        hipLaunchKernelGGL(k_param_final, dim3(nblk(rows, 64)), dim3(64), 0, c->stream, c->n_id, c->n_exp, c->n_alb,
                           c->nchunks, c->partial, c->drot, g->d_alpha, g->d_beta, g->d_delta, g->d_pose);
    }
    if (g->d_lights || g->d_spec || g->d_vertices || g->d_albedo)
        hipLaunchKernelGGL(k_grads_out, dim3(nblk(std::max({V3, (size_t)rr, (size_t)nl3}), 256)), dim3(256), 0,
                           c->stream, G, c->g_vert, nl3, rr, (int)V3, g->d_lights, g->d_spec, g->d_vertices,
                           g->d_albedo);
    ev_record(c, 6);
    HIPCK(c, hipGetLastError());
    c->have_backward = true;
    return FR_OK;
}

static int aov_call(fr_ctx *c, float *out) {
    if (!c) return FR_EINVAL;
    c->err.clear();
    if (!out) return fail(c, FR_EINVAL, "fr_aov: null output");
    if (!c->have_render || !c->records_valid)
        return fail(c, FR_ESTATE, "fr_aov: needs a prior fr_render whose samples fit one chunk");
    Scene S = make_scene(c);
    hipLaunchKernelGGL(k_aov, dim3(nblk((size_t)c->W * c->H, 256)), dim3(256), 0, c->stream, S, c->last_seed, c->last_spp,
                       c->hits, out);
    HIPCK(c, hipGetLastError());
    return FR_OK;
}

static int light_reg_call(fr_ctx *c, const float *lights, float w2, float *grad_lights, float *loss) {
    if (!c) return FR_EINVAL;
    c->err.clear();
    if (!lights) return fail(c, FR_EINVAL, "fr_light_reg: null lights");
    if (!std::isfinite(w2)) return fail(c, FR_EINVAL, "fr_light_reg: non-finite w2");
    hipLaunchKernelGGL(k_light_reg, dim3(1), dim3(64), 0, c->stream, c->nl, lights, w2, grad_lights, loss);
    HIPCK(c, hipGetLastError());
    return FR_OK;
}

static int adam_call(fr_ctx *c, float *param, const float *grad, float *m, float *v, int32_t n, int32_t step,
                     float lr, float beta1, float beta2, float eps) {
    if (!c) return FR_EINVAL;
    c->err.clear();
    if (n < 0 || (n > 0 && (!param || !grad || !m || !v)))
        return fail(c, FR_EINVAL, "fr_adam: null array or negative size");
    if (step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) ||
        !std::isfinite(lr))
        return fail(c, FR_EINVAL, "fr_adam: step >= 1, 0 <= beta < 1, eps > 0, finite lr required");
    if (n == 0) return FR_OK;
    float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, c->stream, n, param, grad, m, v, lr, beta1, beta2,
                       c1, c2, eps);
    HIPCK(c, hipGetLastError());
    return FR_OK;
}

static int loss_l2_call(fr_ctx *c, const float *img, const float *tgt, float *dL, float *loss) {
    if (!c) return FR_EINVAL;
    c->err.clear();
    if (!img || !tgt) return fail(c, FR_EINVAL, "fr_loss_l2: null argument");
    size_t n = (size_t)c->W * c->H * 3;
    int nb = (int)nblk(n, 256);
    hipLaunchKernelGGL(k_loss_partial<256>, dim3(nb), dim3(256), 0, c->stream, n, img, tgt, dL, c->loss_partial);
    if (loss) hipLaunchKernelGGL(k_loss_final<256>, dim3(1), dim3(256), 0, c->stream, nb, c->loss_partial, loss);
    HIPCK(c, hipGetLastError());
    return FR_OK;
}


int fr_blend(fr_ctx *c, const float *alpha, const float *beta, const float *delta, const float *pose,
             float *out_vertices, float *out_albedo) {
    if (!c) return FR_EINVAL;
    if (device_ptrs(c)) return blend_call(c, alpha, beta, delta, pose, out_vertices, out_albedo);
    c->err.clear();
    HostCall h(c, c->io_buf);
    const size_t V3 = 3 * (size_t)c->V;
    const float *a = h.in(alpha, c->n_id), *b = h.in(beta, c->n_exp), *d = h.in(delta, c->n_alb);
    float *ov = h.out(out_vertices, V3), *oa = h.out(out_albedo, V3);
    if (h.err) return h.finish(h.err);
    return h.finish(blend_call(c, a, b, d, pose, ov, oa));
}

int fr_render(fr_ctx *c, const fr_params *p, uint64_t seed, int32_t spp, float *out) {
    if (!c) return FR_EINVAL;
    if (device_ptrs(c) || !p) return render_call(c, p, seed, spp, out);
    c->err.clear();
    HostCall hp(c, c->par_buf), h(c, c->io_buf);
    fr_params q = *p;
    q.alpha = hp.in(p->alpha, c->n_id); q.beta = hp.in(p->beta, c->n_exp); q.delta = hp.in(p->delta, c->n_alb);
    q.lights = hp.in(p->lights, 3 * (size_t)c->nl); q.spec = hp.in(p->spec, (size_t)c->res * c->res);
    float *o = h.out(out, (size_t)c->W * c->H * 3);
    if (hp.err || h.err) return h.finish(hp.err ? hp.err : h.err);
    return h.finish(render_call(c, &q, seed, spp, o));
}

int fr_backward(fr_ctx *c, const float *dLdI, const fr_grads *g) {
    if (!c) return FR_EINVAL;
    if (device_ptrs(c) || !g) return backward_call(c, dLdI, g);
    c->err.clear();
    HostCall h(c, c->io_buf);
    const size_t V3 = 3 * (size_t)c->V;
    const float *dl = h.in(dLdI, (size_t)c->W * c->H * 3);
    fr_grads q;
    q.d_lights = h.out(g->d_lights, 3 * (size_t)c->nl); q.d_spec = h.out(g->d_spec, (size_t)c->res * c->res);
    q.d_vertices = h.out(g->d_vertices, V3); q.d_albedo = h.out(g->d_albedo, V3);
    q.d_alpha = h.out(g->d_alpha, c->n_id); q.d_beta = h.out(g->d_beta, c->n_exp);
    q.d_delta = h.out(g->d_delta, c->n_alb); q.d_pose = h.out(g->d_pose, 6);
    if (h.err) return h.finish(h.err);
    return h.finish(backward_call(c, dl, &q));
}

int fr_aov(fr_ctx *c, float *out) {
    if (!c) return FR_EINVAL;
    if (device_ptrs(c)) return aov_call(c, out);
    c->err.clear();
    HostCall h(c, c->io_buf);
    float *o = h.out(out, (size_t)c->W * c->H * 7);
    if (h.err) return h.finish(h.err);
    return h.finish(aov_call(c, o));
}

int fr_light_reg(fr_ctx *c, const float *lights, float w2, float *grad_lights, float *loss) {
    if (!c) return FR_EINVAL;
    if (device_ptrs(c)) return light_reg_call(c, lights, w2, grad_lights, loss);
    c->err.clear();
    HostCall h(c, c->io_buf);
    const size_t n3 = 3 * (size_t)c->nl;
    const float *l = h.in(lights, n3);
    float *g = h.inout(grad_lights, n3), *ls = h.out(loss, 1);
    if (h.err) return h.finish(h.err);
    return h.finish(light_reg_call(c, l, w2, g, ls));
}

int fr_adam(fr_ctx *c, float *param, const float *grad, float *m, float *v, int32_t n, int32_t step, float lr,
            float beta1, float beta2, float eps) {
    if (!c) return FR_EINVAL;
    if (device_ptrs(c) || n < 0) return adam_call(c, param, grad, m, v, n, step, lr, beta1, beta2, eps);
    c->err.clear();
    HostCall h(c, c->io_buf);
    float *pp = h.inout(param, (size_t)n), *mm = h.inout(m, (size_t)n), *vv = h.inout(v, (size_t)n);
    const float *gg = h.in(grad, (size_t)n);
    if (h.err) return h.finish(h.err);
    return h.finish(adam_call(c, pp, gg, mm, vv, n, step, lr, beta1, beta2, eps));
}

int fr_loss_l2(fr_ctx *c, const float *img, const float *tgt, float *dL, float *loss) {
    if (!c) return FR_EINVAL;
    if (device_ptrs(c)) return loss_l2_call(c, img, tgt, dL, loss);
    c->err.clear();
    HostCall h(c, c->io_buf);
    const size_t n = (size_t)c->W * c->H * 3;
    const float *a = h.in(img, n), *b = h.in(tgt, n);
    float *g = h.out(dL, n), *ls = h.out(loss, 1);
    if (h.err) return h.finish(h.err);
    return h.finish(loss_l2_call(c, a, b, g, ls));
}

int fr_stats(const fr_ctx *cc, fr_stats_t *out) {
    if (!cc || !out) return FR_EINVAL;
    fr_ctx *c = const_cast<fr_ctx *>(cc);   // only its error message is written
    HIPCK(c, hipStreamSynchronize(c->stream));
    std::vector<unsigned long long> all((size_t)kCtrPerKern * kNumKern);
    HIPCK(c, hipMemcpy(all.data(), c->ctr, all.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    memset(out, 0, sizeof *out);
    for (int k = 0; k < kNumKern; ++k) {
        unsigned long long q[8] = {};
        for (int slot = 0; slot < 8; ++slot)
            for (int r = 0; r < kCtrSpread; ++r)
                q[slot] += all[(size_t)k * kCtrPerKern + (size_t)(slot * kCtrSpread + r) * kCtrPad];
        out->rays_camera += q[0]; out->rays_shadow += q[1];
        out->rays_edge_primary += q[2]; out->rays_edge_secondary += q[3];
        out->box_tests += q[4]; out->tri_tests += q[5];
        out->kernel_box_tests[k] = q[4]; out->kernel_tri_tests[k] = q[5];
        out->kernel_rays[k] = q[0] + q[1] + q[2] + q[3];
        out->kernel_shades[k] = q[6];
    }
    out->traversal_overflow = 0;
    if ((c->flags & FR_TIMING) && c->have_render) {
        float t;
        // events of a phase that has not run since the last render are not queried
        if (hipEventElapsedTime(&t, c->ev[0], c->ev[1]) == hipSuccess) out->ms_blend = t;
        if (hipEventElapsedTime(&t, c->ev[1], c->ev[2]) == hipSuccess) out->ms_bvh = t;
        if (hipEventElapsedTime(&t, c->ev[7], c->ev[3]) == hipSuccess) out->ms_edges = t;
        if (hipEventElapsedTime(&t, c->ev[3], c->ev[4]) == hipSuccess) out->ms_render = t;
        for (int k = 0; k < kKernAdj; ++k)
            if (hipEventElapsedTime(&t, c->ev[8 + 2 * k], c->ev[9 + 2 * k]) == hipSuccess) out->ms_kernel[k] = t;
        if (c->have_backward) {
            if (hipEventElapsedTime(&t, c->ev[5], c->ev[6]) == hipSuccess) out->ms_backward = t;
            for (int k = kKernAdj; k < kNumKern; ++k)
                if (hipEventElapsedTime(&t, c->ev[8 + 2 * k], c->ev[9 + 2 * k]) == hipSuccess) out->ms_kernel[k] = t;
        }
        (void)hipGetLastError();   // a failed query must not leak into later calls
    }
    return FR_OK;
}

// ---------------------------------------------- loss without allocation --
// fr_loss_l2_noalloc: the kernels of fr_loss_l2 with their block partials in
// a file-scope device array instead of a context's buffer, so the call needs
// no context and allocates nothing.  Each device the library runs on holds
// its own copy of the array until the process ends.  Host code never uses
// the array's name (on the host it is only a stand-in for the symbol): it
// asks the runtime for the array's address on the current device once, on
// that device's first call, and keeps it per device.
static __device__ __align__(256) double scratch[FR_LOSS_NOALLOC_MAX / 256];

static std::mutex g_scratch_mu;
static double *g_scratch_dev[64];          // per device ordinal
static thread_local std::string g_noctx_err;

static int noctx_fail(int code, const char *msg) {
    g_noctx_err = msg;
    return code;
}

static int scratch_on_current_device(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return noctx_fail(FR_EDEVICE, hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return noctx_fail(FR_EDEVICE, "fr_loss_l2_noalloc: device ordinal above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return noctx_fail(FR_EDEVICE, e != hipSuccess ? hipGetErrorString(e)
                                                                             : "fr_loss_l2_noalloc: null scratch");
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return FR_OK;
}

int fr_loss_l2_noalloc(void *hip_stream, const float *img, const float *tgt, int64_t n, float *dL, float *loss) {
    g_noctx_err.clear();
    if (!img || !tgt) return noctx_fail(FR_EINVAL, "fr_loss_l2_noalloc: null image or target");
    if (n < 1 || n > (int64_t)FR_LOSS_NOALLOC_MAX)
        return noctx_fail(FR_EINVAL, "fr_loss_l2_noalloc: n outside 1 .. FR_LOSS_NOALLOC_MAX (16,777,216)");
    double *part = nullptr;
    int rc = scratch_on_current_device(&part);
    if (rc != FR_OK) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    int nb = (int)nblk((size_t)n, 256);
    hipLaunchKernelGGL(k_loss_partial<256>, dim3(nb), dim3(256), 0, st, (size_t)n, img, tgt, dL, part);
    if (loss) hipLaunchKernelGGL(k_loss_final<256>, dim3(1), dim3(256), 0, st, nb, (const double *)part, loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return noctx_fail(FR_EDEVICE, hipGetErrorString(e));
    return FR_OK;
}

const char *fr_last_error(const fr_ctx *c) {
    if (c) return c->err.c_str();
    return g_noctx_err.empty() ? kNoCtx : g_noctx_err.c_str();
}

void fr_destroy(fr_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
    if (c->side) (void)hipStreamSynchronize(c->side);
    if (c->side2) (void)hipStreamSynchronize(c->side2);
    void *ptrs[] = {c->faces, c->edges, c->vf_off, c->vf_idx, c->mean, c->b_id, c->b_exp, c->alb_mean, c->b_alb, c->uv,
                    c->lgeom, c->sorted_tri, c->leaf_node, c->right, c->escape, c->subs, c->height, c->top, c->top_off, c->nodes, c->tris,
                    c->vmodel, c->vm_d, c->pos, c->nrm, c->nlen, c->alb, c->ew, c->tbl_edge, c->tbl_prefix, c->tbl_n,
                    c->tbl_Q, c->tbl_guide, c->es_wmax, c->es_csum, c->es_ccnt, c->edge_rec, c->edge_pl, c->geo_R, c->samples, c->ctr, c->g_light, c->g_spec, c->g_pos, c->g_nrm, c->g_alb, c->g_N,
                    c->g_vert, c->g_m, c->partial, c->loss_partial, c->hits, c->vis, c->sh_queue, c->sh_cnt, c->pe_q, c->pe_cell_n, c->pe_rec, c->sec_list, c->sec_n, c->pe_samples, c->pe_hits,
                    c->pe_f, c->pe_vis, c->pv_queue, c->pv_aux, c->pv_perm, c->lb.key[0], c->lb.key[1], c->lb.val[0], c->lb.val[1], c->lb.hist,
                    c->lb.bounds, c->lb.child, c->lb.parent, c->lb.first, c->lb.last, c->lb.pre, c->lb.arrive, c->lb.box, c->lb.roots, c->lb.n_roots, c->lb.top_idx, c->lb.n_top, c->lb.top_node};
    for (void *p : ptrs) if (p) (void)hipFree(p);
    for (auto &b : c->io_buf) if (b.first) (void)hipFree(b.first);
    for (auto &b : c->par_buf) if (b.first) (void)hipFree(b.first);
    for (auto &e : c->ev) if (e) (void)hipEventDestroy(e);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->side2) (void)hipStreamDestroy(c->side2);
    for (hipEvent_t e : {c->fork_ev, c->join_ev, c->fork2_ev, c->join2_ev})
        if (e) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"

#include "fr_batch.hpp"
