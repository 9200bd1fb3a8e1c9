// Per-evaluation linear BVH (the default; FR_REFIT contexts refit a fixed shape instead).
//
// Steps, all on the device, from the current triangles:
//   k_lbvh_bounds   box of the triangle centroids (c = ((v0 + v1) + v2) / 3,
//                   fp32), min/max exact, one atomic per block and axis on
//                   order-preserving integer images of the floats;
//   k_lbvh_morton   10 bits per axis of the centroid inside that box,
//                   interleaved into a 30-bit Morton code (Morton 1966),
//                   paired with the triangle index;
//   k_sort_*        stable least-significant-digit radix sort of the codes,
//                   8-bit digits, 4 passes; ties keep triangle order, so the
//                   order is that of the unique keys (code, index);
//   k_lbvh_karras   the hierarchy of Karras (HPG 2012): internal node i of
//                   the F-1 covers a range of sorted leaves found from the
//                   longest common prefix of neighbouring keys (equal keys
//                   compared by index), split where that prefix changes;
//   k_lbvh_layout   depth-first position of every node: 2 * (first leaf of
//                   its range) + (number of left turns from the root), which
//                   counts its ancestors and the nodes of the subtrees to its
//                   left; the escape link is that position plus the subtree
//                   size 2 * leaves - 1;
//   k_lbvh_boxes, k_lbvh_boxes_top
//                   leaf boxes and triangle records, then unions up the tree
//                   (the second child to arrive builds its parent: each
//                   internal node receives exactly two arrivals per build, so
//                   the counters' parity needs no reset), written as 16-byte
//                   nodes in depth-first order.
// The result has the layout and node format the traversal reads, so every
// ray kernel is unchanged.

constexpr int kBoxTile = 1024;      // sorted leaves per block of the box pass
constexpr int kTopSlots = 8192;     // LDS arrival counters of the top pass (global-memory climb)
constexpr int kTopFast = 2048;      // spanning nodes climbed in LDS (128 KiB)

struct LbvhBufs {
    uint32_t *key[2]; int *val[2];      // sort ping-pong
    uint32_t *hist; int nb;             // [256][nb] digit counts per block
    unsigned int *bounds;               // [6] ordered-int min xyz, max xyz
    int *child;                         // [2(F-1)] child ids (internal i, leaf F-1+l)
    int *parent;                        // [2F-1]
    int *first, *last;                  // [F-1] leaf range of internal nodes
    int *pre;                           // [2F-1] depth-first position
    unsigned int *arrive;               // [F-1]
    float *box;                         // [2F-1][6]
    int *roots, *n_roots;               // nodes whose parent spans box tiles
    int *top_idx, *n_top;               // [F-1] LDS slot of a node spanning tiles, or -1
    int *top_node;                      // [F-1] node of each such slot
};

__device__ __forceinline__ unsigned int f2ord(float f) {
    unsigned int u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(unsigned int u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
__device__ __forceinline__ v3 tri_centroid(const float *pos, int V, const int *faces, int f) {
    const int *t = faces + 3 * f;
    v3 a = vpos_raw(pos, V, t[0]), b = vpos_raw(pos, V, t[1]), c = vpos_raw(pos, V, t[2]);
    return mk(((a.x + b.x) + c.x) / 3.0f, ((a.y + b.y) + c.y) / 3.0f, ((a.z + b.z) + c.z) / 3.0f);
}

__device__ __forceinline__ void lbvh_bounds_init_body(unsigned int *bounds) {
    if (threadIdx.x < 3) bounds[threadIdx.x] = 0xffffffffu;
    else if (threadIdx.x < 6) bounds[threadIdx.x] = 0u;
}
// the bounds and the two list counters of the box passes
__global__ __launch_bounds__(64) void k_lbvh_bounds_init(unsigned int *bounds, int *n_top, int *n_roots) {
    lbvh_bounds_init_body(bounds);
    if (threadIdx.x == 8) *n_top = 0;
    if (threadIdx.x == 9) *n_roots = 0;
}

__device__ __forceinline__ void lbvh_bounds_body(int F, const float *__restrict__ pos, int V,
        const int *__restrict__ faces, unsigned int *bounds, int bx) {
    int f = bx * blockDim.x + threadIdx.x;
    unsigned int mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u};
    if (f < F) {
        v3 c = tri_centroid(pos, V, faces, f);
        float cc[3] = {c.x, c.y, c.z};
        for (int a = 0; a < 3; ++a) { mn[a] = f2ord(cc[a]); mx[a] = mn[a]; }
    }
    for (int a = 0; a < 3; ++a)
        for (int off = 32; off > 0; off >>= 1) {
            mn[a] = min(mn[a], (unsigned int)__shfl_xor((int)mn[a], off));
            mx[a] = max(mx[a], (unsigned int)__shfl_xor((int)mx[a], off));
        }
    __shared__ unsigned int s[4][6];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) for (int a = 0; a < 3; ++a) { s[w][a] = mn[a]; s[w][3 + a] = mx[a]; }
    __syncthreads();
    if (threadIdx.x < 6) {
        unsigned int r = s[0][threadIdx.x];
        for (int k = 1; k < (int)(blockDim.x / 64); ++k)
            r = threadIdx.x < 3 ? min(r, s[k][threadIdx.x]) : max(r, s[k][threadIdx.x]);
        if (threadIdx.x < 3) atomicMin(&bounds[threadIdx.x], r); else atomicMax(&bounds[threadIdx.x], r);
    }
}
__global__ __launch_bounds__(256) void k_lbvh_bounds(int F, const float *__restrict__ pos, int V,
        const int *__restrict__ faces, unsigned int *bounds) {
    lbvh_bounds_body(F, pos, V, faces, bounds, blockIdx.x);
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {   // 10 bits -> every third bit
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__device__ __forceinline__ void lbvh_morton_body(int F, const float *__restrict__ pos, int V,
        const int *__restrict__ faces, const unsigned int *__restrict__ bounds, uint32_t *__restrict__ key,
        int *__restrict__ val, int bx) {
    int f = bx * blockDim.x + threadIdx.x;
    if (f >= F) return;
    v3 c = tri_centroid(pos, V, faces, f);
    float cc[3] = {c.x, c.y, c.z};
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        float lo = ord2f(bounds[a]), hi = ord2f(bounds[3 + a]);
        float ext = hi - lo;
        float u = ext > 0.0f ? (cc[a] - lo) / ext : 0.0f;
        int qi = (int)floorf(u * 1024.0f);
        q[a] = (uint32_t)min(1023, max(0, qi));
    }
    key[f] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    val[f] = f;
}
__global__ __launch_bounds__(256) void k_lbvh_morton(int F, const float *__restrict__ pos, int V,
        const int *__restrict__ faces, const unsigned int *__restrict__ bounds, uint32_t *__restrict__ key,
        int *__restrict__ val) {
    lbvh_morton_body(F, pos, V, faces, bounds, key, val, blockIdx.x);
}

// radix sort, 8-bit digit at 'shift'; kSortTile elements per block of 256
constexpr int kSortTile = 1024;
__device__ __forceinline__ void sort_hist_body(int n, int shift, const uint32_t *__restrict__ key,
                                               uint32_t *__restrict__ hist, int nb, int bx) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (int k = 0; k < kSortTile; k += 256) {
        int i = bx * kSortTile + k + threadIdx.x;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nb + bx] = h[threadIdx.x];
}
__global__ __launch_bounds__(256) void k_sort_hist(int n, int shift, const uint32_t *__restrict__ key,
                                                   uint32_t *__restrict__ hist, int nb) {
    sort_hist_body(n, shift, key, hist, nb, blockIdx.x);
}

// exclusive scan of n counts in place, one block of 1024 threads: each
// thread sums a run of consecutive counts, one block-wide scan of the runs'
// sums, then each thread writes its run's offsets (one barrier in all)
__device__ __forceinline__ void scan_u32_body(int n, uint32_t *a) {
    __shared__ uint32_t s_w[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int per = (n + 1023) / 1024, i0 = (int)threadIdx.x * per, i1 = min(n, i0 + per);
    uint32_t sum = 0;
    for (int i = i0; i < i1; ++i) sum += a[i];
    uint32_t inc = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(inc, off);
        if (lane >= off) inc += t;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int k = 0; k < w; ++k) run += s_w[k];
    for (int i = i0; i < i1; ++i) {
        const uint32_t x = a[i];
        a[i] = run;
        run += x;
    }
}
__global__ __launch_bounds__(1024) void k_scan_u32(int n, uint32_t *a) { scan_u32_body(n, a); }

// stable: within a block, elements keep their order (sub-tile, wave, lane)
__device__ __forceinline__ void sort_scatter_body(int n, int shift, const uint32_t *__restrict__ key_in,
        const int *__restrict__ val_in, const uint32_t *__restrict__ offs, int nb, uint32_t *__restrict__ key_out,
        int *__restrict__ val_out, int bx) {
    __shared__ uint32_t cnt[4][256];
    __shared__ uint32_t run[256];       // elements of each digit placed by earlier sub-tiles
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    run[threadIdx.x] = offs[threadIdx.x * nb + bx];
    for (int k = 0; k < kSortTile; k += 256) {
        for (int q = threadIdx.x; q < 4 * 256; q += 256) cnt[q >> 8][q & 255] = 0;
        __syncthreads();
        int i = bx * kSortTile + k + threadIdx.x;
        bool valid = i < n;
        uint32_t kv = valid ? key_in[i] : 0u;
        uint32_t d = (kv >> shift) & 255u;
        unsigned long long same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            unsigned long long m = __ballot((d >> b) & 1u);
            same &= ((d >> b) & 1u) ? m : ~m;
        }
        int rank = __popcll(same & ((1ull << lane) - 1ull));
        if (valid && rank == 0) cnt[w][d] = (uint32_t)__popcll(same);   // group leader
        __syncthreads();
        if (valid) {
            uint32_t before = 0;
            for (int q = 0; q < w; ++q) before += cnt[q][d];
            uint32_t dst = run[d] + before + (uint32_t)rank;
            key_out[dst] = kv;
            val_out[dst] = val_in[i];
        }
        __syncthreads();
        run[threadIdx.x] += cnt[0][threadIdx.x] + cnt[1][threadIdx.x] + cnt[2][threadIdx.x] + cnt[3][threadIdx.x];
        __syncthreads();
    }
}
__global__ __launch_bounds__(256) void k_sort_scatter(int n, int shift, const uint32_t *__restrict__ key_in,
        const int *__restrict__ val_in, const uint32_t *__restrict__ offs, int nb, uint32_t *__restrict__ key_out,
        int *__restrict__ val_out) {
    sort_scatter_body(n, shift, key_in, val_in, offs, nb, key_out, val_out, blockIdx.x);
}

__device__ __forceinline__ int lbvh_delta(const uint32_t *key, int F, int i, int j) {
    if (j < 0 || j >= F) return -1;
    uint32_t a = key[i], b = key[j];
    return a == b ? 32 + __clz((uint32_t)(i ^ j)) : __clz(a ^ b);
}

__device__ __forceinline__ void lbvh_karras_body(int F, const uint32_t *__restrict__ key, int *__restrict__ child,
        int *__restrict__ parent, int *__restrict__ first, int *__restrict__ last, int *__restrict__ top_idx,
        int *__restrict__ n_top, int *__restrict__ top_node, int bx) {
    int i = bx * blockDim.x + threadIdx.x;
    if (i >= F - 1) return;
    int d = lbvh_delta(key, F, i, i + 1) > lbvh_delta(key, F, i, i - 1) ? 1 : -1;
    int dmin = lbvh_delta(key, F, i, i - d);
    int lmax = 2;
    while (lbvh_delta(key, F, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (lbvh_delta(key, F, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = lbvh_delta(key, F, i, j);
    int s = 0, t, k = 2;
    do {
        t = (l + k - 1) / k;
        if (lbvh_delta(key, F, i, i + (s + t) * d) > dnode) s += t;
        k *= 2;
    } while (t > 1);
    int g = i + s * d + min(d, 0);
    int lo = min(i, j), hi = max(i, j);
    int cl = lo == g ? (F - 1) + g : g;
    int cr = hi == g + 1 ? (F - 1) + g + 1 : g + 1;
    child[2 * i] = cl;
    child[2 * i + 1] = cr;
    parent[cl] = i;
    parent[cr] = i;
    first[i] = lo;
    last[i] = hi;
    int slot = -1;
    if (lo / kBoxTile != hi / kBoxTile) {
        slot = atomicAdd(n_top, 1);   // at most F - 1 nodes
        top_node[slot] = i;
    }
    top_idx[i] = slot;
    if (i == 0) parent[0] = -1;
}
__global__ __launch_bounds__(256) void k_lbvh_karras(int F, const uint32_t *__restrict__ key, int *__restrict__ child,
        int *__restrict__ parent, int *__restrict__ first, int *__restrict__ last, int *__restrict__ top_idx,
        int *__restrict__ n_top, int *__restrict__ top_node) {
    lbvh_karras_body(F, key, child, parent, first, last, top_idx, n_top, top_node, blockIdx.x);
}

__device__ __forceinline__ void lbvh_layout_body(int F, const int *__restrict__ child, const int *__restrict__ parent,
        const int *__restrict__ first, int *__restrict__ pre, int bx) {
    int x = bx * blockDim.x + threadIdx.x;
    if (x >= 2 * F - 1) return;
    int a = x >= F - 1 ? x - (F - 1) : first[x];
    int left_turns = 0, cur = x;
    for (int p = (F > 1 ? parent[cur] : -1); p >= 0; cur = p, p = parent[cur])
        if (child[2 * p] == cur) ++left_turns;
    pre[x] = 2 * a + left_turns;
}
__global__ __launch_bounds__(256) void k_lbvh_layout(int F, const int *__restrict__ child, const int *__restrict__ parent,
        const int *__restrict__ first, int *__restrict__ pre) {
    lbvh_layout_body(F, child, parent, first, pre, blockIdx.x);
}

// Boxes bottom-up in two passes without device-wide fences or global
// atomics.  Pass 1: one block per kBoxTile sorted leaves; a leaf's thread
// writes the leaf and climbs while the parent's leaf range lies inside the
// block's range (both children are then this block's), the second arrival
// building the parent.  An internal node's index lies inside its own leaf
// range, so its arrival counter is an LDS word at (index - first leaf of
// the block); workgroup-scope fences order the box writes.  The node where a
// climb stops at a parent spanning blocks goes to a list.  Pass 2: one block
// climbs from the listed nodes through the spanning nodes the same way.
// With at most kTopFast spanning nodes (every face mesh here) the climb runs
// in LDS: each spanning node's slot (assigned by k_lbvh_karras) holds its two
// child boxes, its parent's slot and its node's position and link, all
// loaded at once before the climb, so a climb step costs LDS accesses only
// instead of a chain of dependent global loads.  Past that, the boxes go
// through global memory, with LDS counters at the slots (global ones, whose
// parity needs no reset, past kTopSlots).
__device__ __forceinline__ void lbvh_union_write(int F, int p, const int *child, const int *first, const int *last,
        const int *pre, float *box, Node *nodes) {
    const volatile float *vb = box;
    int cl = child[2 * p], cr = child[2 * p + 1];
    float u[6];
    for (int k = 0; k < 3; ++k) {
        u[k] = fminf(vb[6 * cl + k], vb[6 * cr + k]);
        u[3 + k] = fmaxf(vb[6 * cl + 3 + k], vb[6 * cr + 3 + k]);
    }
    for (int k = 0; k < 6; ++k) box[6 * p + k] = u[k];
    int pp = pre[p];
    nodes[pp] = make_node(u[0], u[1], u[2], u[3], u[4], u[5], pp + 2 * (last[p] - first[p] + 1) - 1);
}

__device__ __forceinline__ void lbvh_boxes_body(int F, const int *__restrict__ faces, const float *__restrict__ pos,
        int V, const int *__restrict__ sorted, const int *__restrict__ child, const int *__restrict__ parent,
        const int *__restrict__ first, const int *__restrict__ last, const int *__restrict__ pre,
        float *box, Node *__restrict__ nodes, float4 *__restrict__ tris, int *__restrict__ roots,
        int *__restrict__ n_roots, int tb) {
    // The climb runs in LDS.  Every internal node inside the block's range
    // has its index in [lo, hi] (an internal node's index lies in its own
    // leaf range), so slot (index - lo) holds its parent, range, children,
    // position and box, loaded at once before the climb, and leaf l's box
    // sits at slot (l - lo).  A climb step then costs LDS accesses only
    // instead of a chain of dependent global loads; only the boxes of the
    // nodes handed to the second pass go to global memory.
    __shared__ int s_par[kBoxTile], s_first[kBoxTile], s_last[kBoxTile], s_cl[kBoxTile], s_cr[kBoxTile],
        s_pre[kBoxTile];
    __shared__ float s_ibox[6 * kBoxTile], s_lbox[6 * kBoxTile];
    __shared__ unsigned int arr[kBoxTile];
    const int lo = tb * kBoxTile, hi = min(F, lo + kBoxTile) - 1;
    const int t = (int)threadIdx.x;
    arr[t] = 0u;
    if (lo + t <= min(hi, F - 2)) {              // internal node lo + t
        const int p = lo + t;
        s_par[t] = parent[p]; s_first[t] = first[p]; s_last[t] = last[p];
        s_cl[t] = child[2 * p]; s_cr[t] = child[2 * p + 1]; s_pre[t] = pre[p];
    }
    const int l = lo + t;
    int x = (F - 1) + l;
    int p = -1;
    if (l < F) {
        const int f = sorted[l];
        const int *tv = faces + 3 * f;
        v3 a = vpos_raw(pos, V, tv[0]), b = vpos_raw(pos, V, tv[1]), c = vpos_raw(pos, V, tv[2]);
        tris[3 * f] = make_float4(a.x, a.y, a.z, b.x);
        tris[3 * f + 1] = make_float4(b.y, b.z, c.x, c.y);
        tris[3 * f + 2] = make_float4(c.z, __int_as_float(f), 0.0f, 0.0f);
        float bx[6] = {fminf(fminf(a.x, b.x), c.x) - kBoxPad, fminf(fminf(a.y, b.y), c.y) - kBoxPad,
                       fminf(fminf(a.z, b.z), c.z) - kBoxPad, fmaxf(fmaxf(a.x, b.x), c.x) + kBoxPad,
                       fmaxf(fmaxf(a.y, b.y), c.y) + kBoxPad, fmaxf(fmaxf(a.z, b.z), c.z) + kBoxPad};
        for (int k = 0; k < 6; ++k) s_lbox[6 * t + k] = bx[k];
        nodes[pre[x]] = make_node(bx[0], bx[1], bx[2], bx[3], bx[4], bx[5], ~f);
        p = F > 1 ? parent[x] : -1;
    }
    __syncthreads();
    if (l >= F) return;
    const float *xb = s_lbox + 6 * t;           // box of x
    for (;;) {
        if (p < 0) return;                                    // x is the root
        if (p < lo || p > hi || s_first[p - lo] < lo || s_last[p - lo] > hi) {   // parent spans blocks
            for (int k = 0; k < 6; ++k) box[6 * x + k] = xb[k];
            roots[atomicAdd(n_roots, 1)] = x;
            return;
        }
        const int sp = p - lo;
        if (atomicAdd(&arr[sp], 1u) == 0u) return;           // first child: the sibling continues
        __threadfence_block();
        const int cl = s_cl[sp], cr = s_cr[sp];
        const float *bl = cl >= F - 1 ? s_lbox + 6 * (cl - (F - 1) - lo) : s_ibox + 6 * (cl - lo);
        const float *br = cr >= F - 1 ? s_lbox + 6 * (cr - (F - 1) - lo) : s_ibox + 6 * (cr - lo);
        float u[6];
        for (int k = 0; k < 3; ++k) {
            u[k] = fminf(bl[k], br[k]);
            u[3 + k] = fmaxf(bl[3 + k], br[3 + k]);
        }
        float *pb = s_ibox + 6 * sp;
        for (int k = 0; k < 6; ++k) pb[k] = u[k];
        const int pp = s_pre[sp];
        nodes[pp] = make_node(u[0], u[1], u[2], u[3], u[4], u[5], pp + 2 * (s_last[sp] - s_first[sp] + 1) - 1);
        __threadfence_block();
        x = p;
        xb = pb;
        p = s_par[sp];
    }
}
__global__ __launch_bounds__(kBoxTile) void k_lbvh_boxes(int F, const int *__restrict__ faces, const float *__restrict__ pos,
        int V, const int *__restrict__ sorted, const int *__restrict__ child, const int *__restrict__ parent,
        const int *__restrict__ first, const int *__restrict__ last, const int *__restrict__ pre,
        float *box, Node *__restrict__ nodes, float4 *__restrict__ tris, int *__restrict__ roots,
        int *__restrict__ n_roots) {
    lbvh_boxes_body(F, faces, pos, V, sorted, child, parent, first, last, pre, box, nodes, tris, roots, n_roots,
                    blockIdx.x);
}

__device__ __forceinline__ void lbvh_boxes_top_body(int F, const int *__restrict__ child,
        const int *__restrict__ parent, const int *__restrict__ first, const int *__restrict__ last,
        const int *__restrict__ pre, const int *__restrict__ top_idx, const int *__restrict__ top_node,
        const int *__restrict__ n_top, unsigned int *__restrict__ arrive, float *box, Node *__restrict__ nodes,
        const int *__restrict__ roots, const int *__restrict__ n_roots) {
    __shared__ float4 smem[kTopFast * 4];
    const int nt = *n_top, nr = *n_roots;
    if (nt <= kTopFast) {
        float *cb = (float *)smem;                          // [slot][2 children][6]
        int *pinfo = (int *)(cb + 12 * kTopFast);           // 2 * parent slot + side, or -1 at the root
        int *pos = pinfo + kTopFast;                        // the node's depth-first position
        int *link = pos + kTopFast;                         // its escape link
        unsigned int *arr = (unsigned int *)(link + kTopFast);
        for (int s = threadIdx.x; s < nt; s += blockDim.x) {
            const int p = top_node[s], q = parent[p], a = pre[p];
            pinfo[s] = q < 0 ? -1 : 2 * top_idx[q] + (child[2 * q] == p ? 0 : 1);
            pos[s] = a;
            link[s] = a + 2 * (last[p] - first[p] + 1) - 1;
            arr[s] = 0u;
        }
        for (int r = threadIdx.x; r < nr; r += blockDim.x) {   // the listed nodes' boxes, done by pass 1
            const int x = roots[r], q = parent[x];
            float *d = cb + 6 * (2 * top_idx[q] + (child[2 * q] == x ? 0 : 1));
            for (int k = 0; k < 6; ++k) d[k] = box[6 * x + k];
        }
        __syncthreads();
        for (int r = threadIdx.x; r < nr; r += blockDim.x) {
            int s = top_idx[parent[roots[r]]];
            for (;;) {
                __threadfence_block();
                if (atomicAdd(&arr[s], 1u) == 0u) break;     // first child: the sibling continues
                __threadfence_block();
                const float *c = cb + 12 * s;
                float u[6];
                for (int k = 0; k < 3; ++k) {
                    u[k] = fminf(c[k], c[6 + k]);
                    u[3 + k] = fmaxf(c[3 + k], c[9 + k]);
                }
                nodes[pos[s]] = make_node(u[0], u[1], u[2], u[3], u[4], u[5], link[s]);
                const int pi = pinfo[s];
                if (pi < 0) break;                             // the tree's root
                for (int k = 0; k < 6; ++k) cb[6 * pi + k] = u[k];
                s = pi >> 1;
            }
        }
        return;
    }
    unsigned int *arr = (unsigned int *)smem;               // kTopSlots counters
    for (int k = threadIdx.x; k < kTopSlots; k += blockDim.x) arr[k] = 0u;
    __syncthreads();
    for (int r = threadIdx.x; r < nr; r += blockDim.x) {
        int x = roots[r];
        for (;;) {
            int p = parent[x];
            if (p < 0) break;
            int ti = top_idx[p];
            unsigned int old = ti < kTopSlots ? atomicAdd(&arr[ti], 1u) : atomicAdd(&arrive[p], 1u);
            if ((old & 1u) == 0u) break;
            __threadfence_block();
            lbvh_union_write(F, p, child, first, last, pre, box, nodes);
            __threadfence_block();
            x = p;
        }
    }
}
__global__ __launch_bounds__(1024) void k_lbvh_boxes_top(int F, const int *__restrict__ child,
        const int *__restrict__ parent, const int *__restrict__ first, const int *__restrict__ last,
        const int *__restrict__ pre, const int *__restrict__ top_idx, const int *__restrict__ top_node,
        const int *__restrict__ n_top, unsigned int *__restrict__ arrive, float *box, Node *__restrict__ nodes,
        const int *__restrict__ roots, const int *__restrict__ n_roots) {
    lbvh_boxes_top_body(F, child, parent, first, last, pre, top_idx, top_node, n_top, arrive, box, nodes, roots,
                        n_roots);
}
