// Batched evaluation: many faces, one launch per kernel for all of them.
//
// A batch holds several contexts (each its own mesh, image size, light stage
// and colours, sample count and parameters) and runs the per-evaluation
// pipeline of fr_render / fr_backward for all of them together.  Every
// kernel's work is a body over block-sized tiles (the same bodies the
// single-context kernels run); one launch covers the tiles of all the
// batch's instances, concatenated instance by instance with the instances in
// order of decreasing sample count (the largest first, so that the tail of
// a launch is made of small tiles).  A block finds its instance by binary
// search over the launch's tile prefix and reads the instance's arguments
// from a descriptor table in device memory.
//
// Launch modes, per kernel kind (fr_batch_set_launch, fr_batch_tune):
//   flat        one block per tile, in order;
//   xcd         one block per tile, the tiles dealt to the eight XCDs in
//               contiguous eighths (the dispatcher issues block b to XCD
//               b mod 8), so that each XCD's L2 serves a few instances at a
//               time instead of all of them.
// The shadow-boundary kind also takes its tile size (samples compacted per
// block: 256 or 512).  Every mode computes the same per-sample values:
// images are bitwise those of single-context renders; gradients differ only
// by the order of their fp64 atomic sums.
//
// The descriptor table has a static part (device pointers and sizes, written
// when the batch is configured for a set of sample counts) and a per-call
// part (seed, pose, parameter and output pointers) written by a kernel whose
// arguments carry it, so that a captured graph holds it by value.

constexpr int kDynPerPut = 4;

struct InstDyn {
    uint64_t seed;
    int spp, terms;
    int want_params, pad;
    PoseArgs P;
    DRotArgs D;
    const float *alpha, *beta, *delta, *lights, *spec;
    float *img;
    const float *dLdI;
    float *d_alpha, *d_beta, *d_delta, *d_pose, *d_lights, *d_spec, *d_vertices, *d_albedo;
};

struct Inst {
    Scene S;                    // S.lrgb and S.spec are set per call
    int n_id, n_exp, n_alb, nchunks, chunk, M;
    long long N;                // camera samples W H spp
    const int *vf_off, *vf_idx;
    const float *mean, *b_id, *b_exp, *alb_mean, *b_alb;
    double *vm_d;
    float *vmodel, *pos, *nrm, *nlen, *alb, *ew;
    int *tbl_edge, *tbl_n, *tbl_guide;
    float4 *edge_rec, *edge_pl;
    uint64_t *tbl_prefix, *tbl_Q;
    Node *nodes;
    float4 *tris;
    LbvhBufs lb;
    HitRec *hits;
    unsigned long long *vis;
    uint32_t *sh_queue, *sh_cnt;      // shadow-ray queue [nl][sh_qcap] and its lengths [nl]
    uint32_t sh_qcap;
    float *samples;
    unsigned long long *ctr;
    uint32_t *sec_list, *sec_n;
    PeSample *pe_samples;
    Hit *pe_hits;
    double *pe_f;
    unsigned long long *pe_vis;
    uint32_t *pv_queue;               // silhouette sides' shadow-ray queue [nl][2 M]
    uint32_t *pv_aux, *pv_perm;       // screen-order sort counters and queue lengths; samples in screen order
    GradBufs G;
    double *g_N;
    float *g_vert, *g_m;
    double *partial;
    InstDyn d;
};

struct DynBlob { InstDyn d[kDynPerPut]; };

__global__ __launch_bounds__(256) void k_put_dyn(DynBlob b, Inst *tab, int first, int count) {
    constexpr int kWords = (int)(sizeof(InstDyn) / 4);
    for (int w = threadIdx.x; w < count * kWords; w += blockDim.x) {
        const int k = w / kWords, o = w - k * kWords;
        reinterpret_cast<uint32_t *>(&tab[first + k].d)[o] = reinterpret_cast<const uint32_t *>(&b.d[k])[o];
    }
    if ((int)threadIdx.x < count) {
        tab[first + threadIdx.x].S.lrgb = b.d[threadIdx.x].lights;
        tab[first + threadIdx.x].S.spec = b.d[threadIdx.x].spec;
    }
}

// ---- kernel kinds: the instance's arguments for each body ---------------
enum {
    bkBlend, bkPose, bkNormals, bkLbvhInit, bkBounds, bkMorton, bkSortHist, bkScan, bkSortScatter, bkKarras,
    bkLayout, bkBoxes, bkBoxesTop, bkEdgeWeights, bkEdgeScan, bkZeroFwd, bkCamera, bkShPropose, bkShTrace, bkShade,
    bkPixelMean,
    bkZeroBwd, bkAdj, bkSecondary, bkSecValue, bkPrimarySetup, bkPvScan, bkPvOrder, bkPvPropose, bkPvTrace, bkPrimaryShade, bkPrimaryScatter,
    bkNormalAdj, bkChainGather, bkParamPartial, bkParamFinal, bkGradOut, bkNum
};
static const char *const kKindName[bkNum] = {
    "blend", "pose", "normals", "lbvh_init", "lbvh_bounds", "lbvh_morton", "sort_hist", "sort_scan", "sort_scatter",
    "lbvh_karras", "lbvh_layout", "lbvh_boxes", "lbvh_boxes_top", "edge_weights", "edge_scan", "zero_fwd",
    "fwd_camera", "sh_propose", "sh_trace", "fwd_shade", "pixel_mean", "zero_bwd", "render_adj", "edge_secondary",
    "edge_secondary_value", "edge_primary_setup", "pv_scan", "pv_order", "pv_propose", "pv_trace", "edge_primary_shade", "edge_primary_scatter",
    "normal_adj", "chain_gather", "param_partial", "param_final", "grad_out"};

#define FR_KIND(NAME, THREADS) struct NAME { static constexpr int kThreads = THREADS; \
    __device__ static void run(const Inst &I, int arg, int bx, int by, int gx)

FR_KIND(KBlend, 64) {
    blend_body(I.S.V, I.n_id, I.n_exp, I.n_alb, I.mean, I.b_id, I.b_exp, I.alb_mean, I.b_alb, I.d.alpha, I.d.beta,
               I.d.delta, I.vm_d, I.vmodel, I.alb, bx, by, I.S.geo_R);
}};
FR_KIND(KPose, 256) { pose_body(I.S.V, I.vm_d, I.d.P, I.pos, bx, I.S.geo_R); }};
FR_KIND(KNormals, 256) { normals_body(I.S.V, I.S.faces, I.vf_off, I.vf_idx, I.pos, I.nrm, I.nlen, bx); }};
FR_KIND(KLbvhInit, 64) {
    lbvh_bounds_init_body(I.lb.bounds);
    if (threadIdx.x == 8) *I.lb.n_top = 0;
    if (threadIdx.x == 9) *I.lb.n_roots = 0;
}};
FR_KIND(KBounds, 256) { lbvh_bounds_body(I.S.F, I.pos, I.S.V, I.S.faces, I.lb.bounds, bx); }};
FR_KIND(KMorton, 256) {
    lbvh_morton_body(I.S.F, I.pos, I.S.V, I.S.faces, I.lb.bounds, I.lb.key[0], I.lb.val[0], bx);
}};
FR_KIND(KSortHist, 256) {   // arg: pass
    sort_hist_body(I.S.F, 8 * arg, I.lb.key[arg & 1], I.lb.hist, I.lb.nb, bx);
}};
FR_KIND(KScan, 1024) { scan_u32_body(256 * I.lb.nb, I.lb.hist); }};
FR_KIND(KSortScatter, 256) {
    const int in = arg & 1;
    sort_scatter_body(I.S.F, 8 * arg, I.lb.key[in], I.lb.val[in], I.lb.hist, I.lb.nb, I.lb.key[in ^ 1],
                      I.lb.val[in ^ 1], bx);
}};
FR_KIND(KKarras, 256) {
    lbvh_karras_body(I.S.F, I.lb.key[0], I.lb.child, I.lb.parent, I.lb.first, I.lb.last, I.lb.top_idx, I.lb.n_top,
                     I.lb.top_node, bx);
}};
FR_KIND(KLayout, 256) { lbvh_layout_body(I.S.F, I.lb.child, I.lb.parent, I.lb.first, I.lb.pre, bx); }};
FR_KIND(KBoxes, kBoxTile) {
    lbvh_boxes_body(I.S.F, I.S.faces, I.pos, I.S.V, I.lb.val[0], I.lb.child, I.lb.parent, I.lb.first, I.lb.last,
                    I.lb.pre, I.lb.box, I.nodes, I.tris, I.lb.roots, I.lb.n_roots, bx);
}};
FR_KIND(KBoxesTop, 1024) {
    lbvh_boxes_top_body(I.S.F, I.lb.child, I.lb.parent, I.lb.first, I.lb.last, I.lb.pre, I.lb.top_idx,
                        I.lb.top_node, I.lb.n_top, I.lb.arrive, I.lb.box, I.nodes, I.lb.roots, I.lb.n_roots);
}};
FR_KIND(KEdgeWeights, 256) { edge_weights_body(I.S, I.S.lgeom, I.ew, I.edge_rec, I.edge_pl, bx); }};
FR_KIND(KEdgeScan, 1024) {
    edge_scan_body<1024>(I.S.E, I.ew, I.tbl_edge, I.tbl_prefix, I.tbl_n, I.tbl_Q, I.tbl_guide, bx);
}};
FR_KIND(KZeroFwd, 64) {
    for (int e = (int)threadIdx.x; e < 8 * kCtrSpread * kKernAdj; e += 64) I.ctr[e * kCtrPad] = 0ull;
    for (int e = (int)threadIdx.x; e < I.S.nl; e += 64) I.sh_cnt[e] = 0u;
}};
FR_KIND(KCamera, kTraceBlock) {
    fwd_camera_body(I.S, I.d.seed, I.d.spp, 0, I.N, I.hits, I.vis, I.ctr + kCtrPerKern * kKernCamera, bx);
}};
FR_KIND(KShPropose, 256) {
    sh_propose_all_body(I.S, I.d.seed, 0, I.N, I.hits, I.sh_queue, I.sh_qcap, I.sh_cnt,
                        I.ctr + kCtrPerKern * kKernShadow, bx);
}};
FR_KIND(KShTrace, kTraceBlock) {
    sh_trace_body(I.S, I.d.seed, 0, I.hits, I.sh_queue, I.sh_qcap, I.sh_cnt, I.vis, I.ctr + kCtrPerKern * kKernShadow,
                  bx, by);
}};
FR_KIND(KShade, 256) {
    fwd_shade_body(I.S, I.d.seed, I.d.spp, 0, I.N, I.hits, I.vis, I.samples, I.ctr + kCtrPerKern * kKernShade, bx);
}};
FR_KIND(KPixelMean, 256) { pixel_mean_body(I.M, I.d.spp, I.samples, I.d.img, bx); }};
FR_KIND(KZeroBwd, 256) {
    const int i = bx * 256 + threadIdx.x, V3 = 3 * I.S.V;
    if (i < 3 * I.S.nl) I.G.d_light[i] = 0.0;
    if (i < I.S.res * I.S.res) I.G.d_spec[i] = 0.0;
    if (i < V3) { I.G.d_pos[i] = 0.0; I.G.d_nrm[i] = 0.0; I.G.d_alb[i] = 0.0; }
    if (i < 8 * kCtrSpread * (kNumKern - kKernAdj)) I.ctr[(8 * kCtrSpread * kKernAdj + i) * kCtrPad] = 0ull;
    if (i == 0) *I.sec_n = 0u;
    if (i < pv_aux_len(I.S.W, I.S.H, I.S.nl)) I.pv_aux[i] = 0u;
}};
FR_KIND(KAdj, 256) {
    if (!(I.d.terms & FR_TERM_INTERIOR)) return;
    render_adj_body(I.S, I.d.seed, I.d.spp, 0, I.N, I.d.dLdI, I.G, I.hits, I.vis, I.ctr + kCtrPerKern * kKernAdj, bx);
}};
template <int TS> FR_KIND(KSecondary, 256) {
    if (!(I.d.terms & FR_TERM_SECONDARY)) return;
    edge_secondary_body<TS>(I.S, I.d.seed, I.d.spp, 0, I.N, I.d.dLdI, I.hits, I.sec_list, I.sec_n,
                            I.ctr + kCtrPerKern * kKernSecondary, bx, by);
}};
FR_KIND(KSecValue, 256) {
    if (!(I.d.terms & FR_TERM_SECONDARY)) return;
    edge_secondary_value_body(I.S, I.d.seed, I.d.spp, 0, I.d.dLdI, I.hits, I.sec_list, I.sec_n, I.G.d_pos, bx, gx);
}};
FR_KIND(KPrimarySetup, kTraceBlock) {
    if (!(I.d.terms & FR_TERM_PRIMARY)) return;
    edge_primary_setup_body(I.S, I.d.seed, I.M, I.pe_samples, I.pe_hits, I.pe_vis, I.pv_aux,
                            I.ctr + kCtrPerKern * kKernPrimary, bx);
}};
FR_KIND(KPvScan, 1024) {
    if (!(I.d.terms & FR_TERM_PRIMARY)) return;
    scan_u32_body(pv_keys(I.S.W, I.S.H), I.pv_aux);
}};
FR_KIND(KPvOrder, 256) {
    if (!(I.d.terms & FR_TERM_PRIMARY)) return;
    pv_order_body(I.S, I.M, I.pe_samples, I.pv_aux, I.pv_perm, bx);
}};
FR_KIND(KPvPropose, 256) {
    if (!(I.d.terms & FR_TERM_PRIMARY)) return;
    pv_propose_body(I.S, I.d.seed, I.pe_samples, I.pe_hits, I.pv_perm, I.pv_aux, I.pv_queue, 2 * (uint32_t)I.M,
                    I.ctr + kCtrPerKern * kKernPrimary, bx);
}};
FR_KIND(KPvTrace, kTraceBlock) {
    if (!(I.d.terms & FR_TERM_PRIMARY)) return;
    pv_trace_body(I.S, I.d.seed, I.pe_samples, I.pe_hits, I.pv_queue, 2 * (uint32_t)I.M,
                  I.pv_aux + 2 * pv_keys(I.S.W, I.S.H), I.pe_vis, I.ctr + kCtrPerKern * kKernPrimary, bx, by);
}};
FR_KIND(KPrimaryShade, 256) {
    if (!(I.d.terms & FR_TERM_PRIMARY)) return;
    edge_primary_shade_body(I.S, I.d.seed, I.M, I.pe_samples, I.pe_hits, I.pe_vis, I.pe_f, I.ctr + kCtrPerKern * kKernPrimary, bx);
}};
FR_KIND(KPrimaryScatter, 256) {
    if (!(I.d.terms & FR_TERM_PRIMARY)) return;
    edge_primary_scatter_body(I.S, I.M, I.d.dLdI, I.pe_samples, I.pe_f, I.G.d_pos, bx);
}};
FR_KIND(KNormalAdj, 256) { normal_adj_body(I.S.V, I.nrm, I.nlen, I.G.d_nrm, I.g_N, bx); }};
FR_KIND(KChainGather, 256) {
    chain_gather_body(I.S.V, I.S.faces, I.vf_off, I.vf_idx, I.pos, I.g_N, I.G.d_pos, I.d.P, I.g_vert, I.g_m, bx);
}};
FR_KIND(KParamPartial, 256) {
    if (!I.d.want_params) return;
    param_partial_body<256>(I.S.V, I.n_id, I.n_exp, I.n_alb, I.chunk, I.b_id, I.b_exp, I.b_alb, I.g_m, I.G.d_alb,
                            I.g_vert, I.vmodel, I.partial, bx, by, I.nchunks);
}};
FR_KIND(KParamFinal, 64) {
    if (!I.d.want_params) return;
    param_final_body(I.n_id, I.n_exp, I.n_alb, I.nchunks, I.partial, I.d.D, I.d.d_alpha, I.d.d_beta, I.d.d_delta,
                     I.d.d_pose, bx);
}};
FR_KIND(KGradOut, 256) {
    const int i = bx * 256 + threadIdx.x, V3 = 3 * I.S.V;
    if (I.d.d_lights && i < 3 * I.S.nl) I.d.d_lights[i] = (float)I.G.d_light[i];
    if (I.d.d_spec && i < I.S.res * I.S.res) I.d.d_spec[i] = (float)I.G.d_spec[i];
    if (I.d.d_vertices && i < V3) I.d.d_vertices[i] = I.g_vert[i];
    if (I.d.d_albedo && i < V3) I.d.d_albedo[i] = (float)I.G.d_alb[i];
}};
#undef FR_KIND

// ---- the launcher --------------------------------------------------------
struct TileMap {
    const int *pre;           // [n + 1] first tile of each slot
    const int *inst;          // [n] instance of each slot
    const int *gx;            // [n] tiles along x of each slot's instance
    int n, total;
    int xcd;                  // tiles grouped by XCD
};

template <class K>
__device__ __forceinline__ void run_tile(const Inst *__restrict__ tab, const TileMap &m, int arg, int t) {
    int lo = 0, hi = m.n - 1;   // last slot whose first tile is <= t (it is not empty)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (m.pre[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int tl = t - m.pre[lo], gx = m.gx[lo];
    K::run(tab[m.inst[lo]], arg, tl % gx, tl / gx, gx);
}

// One block per tile.  The grid is two-dimensional, rows of kRowTiles
// blocks (the tile is the block's linear index; a dispatch's work-item
// count per dimension must fit in 32 bits, and one row of a batch of many
// large instances would not), and the last row's extra blocks exit.
constexpr unsigned kRowTiles = 65536;
template <class K>
__global__ __launch_bounds__(K::kThreads) void k_multi(const Inst *__restrict__ tab, TileMap m, int arg) {
    int t = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (t >= m.total) return;
    if (m.xcd) {
        const int x = t & 7, k = t >> 3, q = m.total >> 3, r = m.total & 7;
        t = x * q + min(x, r) + k;
    }
    run_tile<K>(tab, m, arg, t);
}

// ====================================================================== //
//                               host side                                //
// ====================================================================== //

static const int kTiles[2] = {256, 512};

static bool kind_tiled(int k) { return k == bkSecondary; }
static bool kind_tunable(int k) {
    return k == bkCamera || k == bkShPropose || k == bkShTrace || k == bkShade || k == bkAdj || k == bkSecondary || k == bkSecValue ||
           k == bkPrimarySetup || k == bkPvPropose || k == bkPvTrace || k == bkPrimaryShade;
}

struct KindPlan { int off, n, total; };

struct fr_batch {
    std::string err;
    int n = 0;
    std::vector<fr_ctx *> ctx;
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    Inst *tab = nullptr;                  // device [n]
    std::vector<Inst> host;               // mirror of the static part
    std::vector<InstDyn> dyn;             // mirror of the per-call part
    std::vector<int> spp;                 // configured sample counts (empty: none)
    std::vector<long long> N;
    std::vector<char> solo;               // instances above one chunk: their context's own path
    std::vector<int> order;               // slots: instances by decreasing N
    std::vector<uint64_t> gen;            // contexts' render generations after the last batch render
    fr_launch launch[bkNum];
    int *plan = nullptr; size_t plan_cap = 0;
    KindPlan kp[bkNum];
    bool plan_dirty = true;
    size_t lds_res2 = 0, lds_adj = 0;     // dynamic LDS bytes
    bool capturing = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[2 * bkNum + 6] = {};   // per kind; render, backward; the tuner's replays
    bool timed[bkNum] = {};
    float ms[bkNum] = {};
    float ms_render = 0, ms_backward = 0;
    bool have_render = false, have_backward = false;
};

static int bfail(fr_batch *b, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    return code;
}

#define BHIPCK(b, call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return bfail((b), e_ == hipErrorOutOfMemory ? FR_ENOMEM : FR_EDEVICE, "%s: %s (%s:%d)", #call, \
                         hipGetErrorString(e_), __FILE__, __LINE__);                     \
    } while (0)

static int kind_threads(int k) {
    switch (k) {
    case bkBlend: case bkLbvhInit: case bkZeroFwd: case bkParamFinal: return 64;
    case bkScan: case bkBoxes: case bkBoxesTop: case bkEdgeScan: case bkPvScan: return 1024;
    default: return 256;
    }
}

// tiles of kind k for instance i: gx along x, gy along y (bodies see bx, by)
static void kind_grid(const fr_batch *b, int k, int i, int &gx, int &gy) {
    const fr_ctx *c = b->ctx[i];
    const long long N = b->N[i];
    const int V = c->V, F = c->F, nl = c->nl, M = c->W * c->H, rr = c->res * c->res;
    const int rows = c->n_id + c->n_exp + c->n_alb + 12;
    const int ts = b->launch[k].tile;
    gy = 1;
    if (b->solo[i]) { gx = 0; return; }      // no tiles: rendered on its own
    switch (k) {
    case bkBlend: gx = (int)nblk(V, 64); gy = 6; break;
    case bkPose: case bkNormals: case bkNormalAdj: case bkChainGather: gx = (int)nblk(V, 256); break;
    case bkLbvhInit: case bkScan: case bkZeroFwd: case bkPvScan: gx = 1; break;
    case bkBounds: case bkMorton: gx = (int)nblk(F, 256); break;
    case bkSortHist: case bkSortScatter: gx = c->lb.nb; break;
    case bkKarras: gx = F > 1 ? (int)nblk(F - 1, 256) : 0; break;
    case bkLayout: gx = (int)nblk(2 * (size_t)F - 1, 256); break;
    case bkBoxes: gx = (int)nblk(F, kBoxTile); break;
    case bkBoxesTop: gx = F > 1 ? 1 : 0; break;
    case bkEdgeWeights: gx = (int)nblk(c->E, 256); break;
    case bkEdgeScan: gx = 1 + nl; break;
    case bkCamera: gx = (int)nblk(N, kTraceBlock); break;
    case bkShade: case bkAdj: gx = (int)nblk(N, 256); break;
    case bkSecondary: gx = (int)nblk(N, ts); gy = sec_light_groups(nl); break;
    case bkShPropose: gx = (int)nblk(N, 256); break;
    case bkShTrace: gx = (int)nblk(N, kTraceBlock); gy = nl; break;
    case bkPrimarySetup: gx = (int)nblk(M, kTraceBlock); break;
    case bkPixelMean: case bkPvOrder: case bkPrimaryScatter: gx = (int)nblk(M, 256); break;
    case bkZeroBwd:
        gx = (int)nblk(std::max({3 * V, rr, 3 * nl, 8 * kCtrSpread * kNumKern, pv_aux_len(c->W, c->H, nl)}), 256);
        break;
    case bkSecValue: gx = (int)std::min<long long>(1024, std::max<long long>(1, (N + 1023) / 1024)); break;
    case bkPvPropose: gx = (int)nblk(2 * (size_t)M, 256); break;
    case bkPvTrace: gx = (int)nblk(2 * (size_t)M, kTraceBlock); gy = nl; break;
    case bkPrimaryShade: gx = (int)nblk(2 * (size_t)M, 256); break;
    case bkParamPartial: gx = rows; gy = c->nchunks; break;
    case bkParamFinal: gx = (int)nblk(rows, 64); break;
    case bkGradOut: gx = (int)nblk(std::max({3 * V, rr, 3 * nl}), 256); break;
    default: gx = 0;
    }
}

static int build_plan(fr_batch *b) {
    // batched work already enqueued reads the current plan: let it finish
    // before the host overwrites it
    BHIPCK(b, hipStreamSynchronize(b->stream));
    std::vector<int> h;
    for (int k = 0; k < bkNum; ++k) {
        KindPlan &p = b->kp[k];
        p.off = (int)h.size();
        p.n = b->n;
        std::vector<int> pre(b->n + 1, 0), inst(b->n), gxs(b->n);
        long long total = 0;
        for (int s = 0; s < b->n; ++s) {
            int i = b->order[s], gx, gy;
            kind_grid(b, k, i, gx, gy);
            pre[s] = (int)total;
            inst[s] = i;
            gxs[s] = std::max(gx, 1);
            total += (long long)gx * gy;
        }
        if (total >= (1ll << 31)) return bfail(b, FR_EINVAL, "fr_batch: kind %s has too many tiles", kKindName[k]);
        pre[b->n] = (int)total;
        p.total = (int)total;
        h.insert(h.end(), pre.begin(), pre.end());
        h.insert(h.end(), inst.begin(), inst.end());
        h.insert(h.end(), gxs.begin(), gxs.end());
    }
    if (h.size() > b->plan_cap) {
        if (b->plan) (void)hipFree(b->plan);
        b->plan = nullptr; b->plan_cap = 0;
        BHIPCK(b, hipMalloc((void **)&b->plan, h.size() * sizeof(int)));
        b->plan_cap = h.size();
    }
    BHIPCK(b, hipMemcpy(b->plan, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
    b->plan_dirty = false;
    return FR_OK;
}

template <class K>
static void launch_k(fr_batch *b, const TileMap &m, int arg, unsigned grid, size_t lds) {
    const unsigned gx = std::min(grid, kRowTiles), gy = (grid + kRowTiles - 1) / kRowTiles;
    hipLaunchKernelGGL(k_multi<K>, dim3(gx, gy), dim3(K::kThreads), lds, b->stream, b->tab, m, arg);
}

static void launch_kind(fr_batch *b, int k, int arg = 0) {
    const KindPlan &p = b->kp[k];
    if (p.total == 0) return;
    const fr_launch &L = b->launch[k];
    TileMap m;
    m.pre = b->plan + p.off;
    m.inst = m.pre + p.n + 1;
    m.gx = m.inst + p.n;
    m.n = p.n;
    m.total = p.total;
    m.xcd = L.mode == FR_LAUNCH_XCD;
    const unsigned grid = (unsigned)p.total;
    const bool tm = (b->flags & FR_TIMING) && !b->capturing;
    if (tm && !b->timed[k]) (void)hipEventRecord(b->ev[2 * k], b->stream);
    const int ts = L.tile;
    switch (k) {
    case bkBlend: launch_k<KBlend>(b, m, arg, grid, 0); break;
    case bkPose: launch_k<KPose>(b, m, arg, grid, 0); break;
    case bkNormals: launch_k<KNormals>(b, m, arg, grid, 0); break;
    case bkLbvhInit: launch_k<KLbvhInit>(b, m, arg, grid, 0); break;
    case bkBounds: launch_k<KBounds>(b, m, arg, grid, 0); break;
    case bkMorton: launch_k<KMorton>(b, m, arg, grid, 0); break;
    case bkSortHist: launch_k<KSortHist>(b, m, arg, grid, 0); break;
    case bkScan: launch_k<KScan>(b, m, arg, grid, 0); break;
    case bkSortScatter: launch_k<KSortScatter>(b, m, arg, grid, 0); break;
    case bkKarras: launch_k<KKarras>(b, m, arg, grid, 0); break;
    case bkLayout: launch_k<KLayout>(b, m, arg, grid, 0); break;
    case bkBoxes: launch_k<KBoxes>(b, m, arg, grid, 0); break;
    case bkBoxesTop: launch_k<KBoxesTop>(b, m, arg, grid, 0); break;
    case bkEdgeWeights: launch_k<KEdgeWeights>(b, m, arg, grid, 0); break;
    case bkEdgeScan: launch_k<KEdgeScan>(b, m, arg, grid, 0); break;
    case bkZeroFwd: launch_k<KZeroFwd>(b, m, arg, grid, 0); break;
    case bkCamera: launch_k<KCamera>(b, m, arg, grid, 0); break;
    case bkShPropose: launch_k<KShPropose>(b, m, arg, grid, 0); break;
    case bkShTrace: launch_k<KShTrace>(b, m, arg, grid, 0);
        break;
    case bkShade: launch_k<KShade>(b, m, arg, grid, b->lds_res2); break;
    case bkPixelMean: launch_k<KPixelMean>(b, m, arg, grid, 0); break;
    case bkZeroBwd: launch_k<KZeroBwd>(b, m, arg, grid, 0); break;
    case bkAdj: launch_k<KAdj>(b, m, arg, grid, b->lds_adj); break;
    case bkSecondary:
        if (ts == 256) launch_k<KSecondary<256>>(b, m, arg, grid, 0);
        else launch_k<KSecondary<512>>(b, m, arg, grid, 0);
        break;
    case bkSecValue: launch_k<KSecValue>(b, m, arg, grid, b->lds_res2); break;
    case bkPrimarySetup: launch_k<KPrimarySetup>(b, m, arg, grid, 0); break;
    case bkPvPropose: launch_k<KPvPropose>(b, m, arg, grid, 0); break;
    case bkPvTrace: launch_k<KPvTrace>(b, m, arg, grid, 0); break;
    case bkPvScan: launch_k<KPvScan>(b, m, arg, grid, 0); break;
    case bkPvOrder: launch_k<KPvOrder>(b, m, arg, grid, 0); break;
    case bkPrimaryShade: launch_k<KPrimaryShade>(b, m, arg, grid, b->lds_res2); break;
    case bkPrimaryScatter: launch_k<KPrimaryScatter>(b, m, arg, grid, 0); break;
    case bkNormalAdj: launch_k<KNormalAdj>(b, m, arg, grid, 0); break;
    case bkChainGather: launch_k<KChainGather>(b, m, arg, grid, 0); break;
    case bkParamPartial: launch_k<KParamPartial>(b, m, arg, grid, 0); break;
    case bkParamFinal: launch_k<KParamFinal>(b, m, arg, grid, 0); break;
    case bkGradOut: launch_k<KGradOut>(b, m, arg, grid, 0); break;
    }
    if (tm) { (void)hipEventRecord(b->ev[2 * k + 1], b->stream); b->timed[k] = true; }
}

// per-call part of the descriptors, carried by kernel arguments
static void put_dyn(fr_batch *b) {
    for (int first = 0; first < b->n; first += kDynPerPut) {
        DynBlob blob;
        memset(&blob, 0, sizeof blob);
        int cnt = std::min(kDynPerPut, b->n - first);
        for (int k = 0; k < cnt; ++k) blob.d[k] = b->dyn[first + k];
        hipLaunchKernelGGL(k_put_dyn, dim3(1), dim3(256), 0, b->stream, blob, b->tab, first, cnt);
    }
}

// timing restarts for the call's kinds
static void begin_call(fr_batch *b, int k0, int k1) {
    for (int k = k0; k <= k1; ++k) b->timed[k] = false;
}

// the evaluation, in the order of fr_render
static void seq_forward(fr_batch *b) {
    begin_call(b, bkBlend, bkPixelMean);
    launch_kind(b, bkBlend);
    launch_kind(b, bkPose);
    launch_kind(b, bkNormals);
    launch_kind(b, bkLbvhInit);
    launch_kind(b, bkBounds);
    launch_kind(b, bkMorton);
    for (int pass = 0; pass < 4; ++pass) {
        launch_kind(b, bkSortHist, pass);
        launch_kind(b, bkScan, pass);
        launch_kind(b, bkSortScatter, pass);
    }
    launch_kind(b, bkKarras);
    launch_kind(b, bkLayout);
    launch_kind(b, bkBoxes);
    launch_kind(b, bkBoxesTop);
    launch_kind(b, bkEdgeWeights);
    launch_kind(b, bkEdgeScan);
    launch_kind(b, bkZeroFwd);
    launch_kind(b, bkCamera);
    launch_kind(b, bkShPropose);
    launch_kind(b, bkShTrace);
    launch_kind(b, bkShade);
    launch_kind(b, bkPixelMean);
}

// the adjoint, in the order of fr_backward
static void seq_backward(fr_batch *b) {
    begin_call(b, bkZeroBwd, bkGradOut);
    for (int k = bkZeroBwd; k <= bkGradOut; ++k) launch_kind(b, k);
}

// buffers sized for the sample counts, static descriptors, tile plan
static int configure(fr_batch *b, const int32_t *spp) {
    if (b->capturing) return bfail(b, FR_ESTATE, "fr_batch: sample counts changed during graph capture");
    // batched work already enqueued reads the descriptor table and the
    // contexts' scratch: let it finish before either changes
    BHIPCK(b, hipStreamSynchronize(b->stream));
    b->spp.assign(spp, spp + b->n);
    b->N.resize(b->n);
    b->host.resize(b->n);
    b->lds_res2 = b->lds_adj = 0;
    b->solo.assign(b->n, 0);
    for (int i = 0; i < b->n; ++i) {
        fr_ctx *c = b->ctx[i];
        const long long N = (long long)c->W * c->H * spp[i];
        b->N[i] = N;
        Inst &I = b->host[i];
        memset(&I, 0, sizeof I);
        if (N > FR_CHUNK_MAX) {      // its own path sizes its scratch on its first render
            b->solo[i] = 1;
            continue;
        }
        if ((size_t)N * 3 > c->samples_cap) {
            if (c->samples) (void)hipFree(c->samples);
            c->samples = nullptr; c->samples_cap = 0;
            BHIPCK(b, hipMalloc((void **)&c->samples, (size_t)N * 3 * sizeof(float)));
            c->samples_cap = (size_t)N * 3;
        }
        if ((size_t)N > c->rec_cap) {
            if (c->hits) (void)hipFree(c->hits);
            if (c->vis) (void)hipFree(c->vis);
            c->hits = nullptr; c->vis = nullptr; c->rec_cap = 0;
            BHIPCK(b, hipMalloc((void **)&c->hits, (size_t)N * sizeof(HitRec)));
            BHIPCK(b, hipMalloc((void **)&c->vis, (size_t)N * sizeof(unsigned long long)));
            c->rec_cap = (size_t)N;
        }
        if ((size_t)N > c->sh_cap) {
            if (c->sh_queue) (void)hipFree(c->sh_queue);
            c->sh_queue = nullptr; c->sh_cap = 0;
            BHIPCK(b, hipMalloc((void **)&c->sh_queue, (size_t)N * c->nl * sizeof(uint32_t)));
            c->sh_cap = (size_t)N;
        }
        const size_t sec = (size_t)N * c->nl;     // every (sample, light) pair at most once
        if (sec > c->sec_cap) {
            if (c->sec_list) (void)hipFree(c->sec_list);
            c->sec_list = nullptr; c->sec_cap = 0;
            BHIPCK(b, hipMalloc((void **)&c->sec_list, sec * sizeof(uint32_t)));
            c->sec_cap = sec;
        }
        c->records_valid = false;
        c->have_render = false;
        I.S = make_scene(c);
        I.n_id = c->n_id; I.n_exp = c->n_exp; I.n_alb = c->n_alb;
        I.nchunks = c->nchunks; I.chunk = c->chunk; I.M = c->W * c->H;
        I.N = N;
        I.vf_off = c->vf_off; I.vf_idx = c->vf_idx;
        I.mean = c->mean; I.b_id = c->b_id; I.b_exp = c->b_exp; I.alb_mean = c->alb_mean; I.b_alb = c->b_alb;
        I.vm_d = c->vm_d; I.vmodel = c->vmodel; I.pos = c->pos; I.nrm = c->nrm; I.nlen = c->nlen; I.alb = c->alb;
        I.ew = c->ew; I.edge_rec = c->edge_rec; I.edge_pl = c->edge_pl;
        I.tbl_edge = c->tbl_edge; I.tbl_n = c->tbl_n; I.tbl_prefix = c->tbl_prefix; I.tbl_Q = c->tbl_Q;
        I.tbl_guide = c->tbl_guide;
        I.nodes = c->nodes; I.tris = c->tris;
        I.lb = c->lb;
        I.hits = c->hits; I.vis = c->vis; I.samples = c->samples; I.ctr = c->ctr;
        I.sh_queue = c->sh_queue; I.sh_cnt = c->sh_cnt; I.sh_qcap = (uint32_t)c->sh_cap;
        I.sec_list = c->sec_list; I.sec_n = c->sec_n;
        I.pe_samples = c->pe_samples; I.pe_hits = c->pe_hits; I.pe_f = c->pe_f; I.pe_vis = c->pe_vis;
        I.pv_queue = c->pv_queue; I.pv_aux = c->pv_aux; I.pv_perm = c->pv_perm;
        I.G = GradBufs{c->g_light, c->g_spec, c->g_pos, c->g_nrm, c->g_alb};
        I.g_N = c->g_N; I.g_vert = c->g_vert; I.g_m = c->g_m; I.partial = c->partial;
        const size_t rr = (size_t)c->res * c->res;
        b->lds_res2 = std::max(b->lds_res2, rr * sizeof(float));
        b->lds_adj = std::max(b->lds_adj, (2 * rr + (size_t)kLightCopies * light_stride(c->nl)) * sizeof(float));
    }
    b->order.resize(b->n);
    for (int i = 0; i < b->n; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return b->N[x] > b->N[y]; });
    for (int i = 0; i < b->n; ++i) b->host[i].d = b->dyn[i];   // the per-call part as the last call left it
    BHIPCK(b, hipMemcpy(b->tab, b->host.data(), sizeof(Inst) * b->n, hipMemcpyHostToDevice));
    b->plan_dirty = true;
    b->have_render = b->have_backward = false;
    return FR_OK;
}

// An instance above one chunk (W*H*spp > FR_CHUNK_MAX) goes through its
// context's own render or adjoint on the batch's stream, after the batched
// kinds: chunk by chunk, the adjoint recomputing each chunk's records.  Its
// scratch is sized by its first render, so a capture after that allocates
// nothing; inside a capture its timing events are left out, since a graph
// keeps no timing.
template <class F>
static int solo_call(fr_batch *b, int i, F f) {
    fr_ctx *c = b->ctx[i];
    const uint32_t flags = c->flags;
    if (b->capturing) c->flags &= ~FR_TIMING;
    const int r = f(c);
    c->flags = flags;
    return r ? bfail(b, r, "instance %d: %s", i, c->err.c_str()) : FR_OK;
}

extern "C" {

int32_t fr_batch_num_kinds(void) { return bkNum; }
const char *fr_batch_kind_name(int32_t kind) { return kind >= 0 && kind < bkNum ? kKindName[kind] : nullptr; }

int fr_batch_create(int32_t n, fr_ctx *const *ctx, uint32_t flags, fr_batch **out) {
    if (!out) return FR_EINVAL;
    *out = nullptr;
    if (n < 1 || n > 4096 || !ctx || (flags & ~FR_TIMING)) return FR_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!ctx[i] || (ctx[i]->flags & FR_REFIT) || !(ctx[i]->flags & FR_DEVICE_PTRS)) return FR_EINVAL;
        for (int k = 0; k < i; ++k)
            if (ctx[k] == ctx[i]) return FR_EINVAL;
    }
    fr_batch *b = new fr_batch();
    b->n = n;
    b->ctx.assign(ctx, ctx + n);
    b->flags = flags;
    b->dyn.assign(n, InstDyn{});
    b->gen.assign(n, 0);
    for (int k = 0; k < bkNum; ++k)
        b->launch[k] = fr_launch{FR_LAUNCH_FLAT, k == bkSecondary ? kSecTile : 0};
    b->stream = ctx[0]->stream;
    if (hipMalloc((void **)&b->tab, sizeof(Inst) * n) != hipSuccess) {
        fr_batch_destroy(b);
        return FR_ENOMEM;
    }
    if (flags & FR_TIMING)
        for (auto &e : b->ev) (void)hipEventCreate(&e);
    *out = b;
    return FR_OK;
}

int fr_batch_set_stream(fr_batch *b, void *stream) {
    if (!b) return FR_EINVAL;
    if (b->capturing && (hipStream_t)stream != b->stream)
        return bfail(b, FR_ESTATE, "fr_batch_set_stream: graph capture in progress");
    b->stream = (hipStream_t)stream;
    for (fr_ctx *c : b->ctx) c->stream = (hipStream_t)stream;
    return FR_OK;
}

int fr_batch_get_launch(const fr_batch *b, int32_t kind, fr_launch *out) {
    if (!b || !out || kind < 0 || kind >= bkNum) return FR_EINVAL;
    *out = b->launch[kind];
    return FR_OK;
}

int fr_batch_set_launch(fr_batch *b, int32_t kind, const fr_launch *l) {
    if (!b) return FR_EINVAL;
    b->err.clear();
    if (!l || kind < 0 || kind >= bkNum) return bfail(b, FR_EINVAL, "fr_batch_set_launch: bad kind or null");
    if (b->capturing) return bfail(b, FR_ESTATE, "fr_batch_set_launch: graph capture in progress");
    if (l->mode != FR_LAUNCH_FLAT && l->mode != FR_LAUNCH_XCD)
        return bfail(b, FR_EINVAL, "fr_batch_set_launch: mode %d is neither FR_LAUNCH_FLAT nor FR_LAUNCH_XCD",
                     l->mode);
    fr_launch v = *l;
    if (kind_tiled(kind)) {
        if (v.tile != 256 && v.tile != 512)
            return bfail(b, FR_EINVAL, "fr_batch_set_launch: tile %d not in {256, 512}", v.tile);
    } else if (v.tile != 0) {
        return bfail(b, FR_EINVAL, "fr_batch_set_launch: kind %s takes no tile size (pass 0)", kKindName[kind]);
    }
    if (kind_tiled(kind) && v.tile != b->launch[kind].tile) b->plan_dirty = true;
    b->launch[kind] = v;
    return FR_OK;
}

int fr_batch_render(fr_batch *b, const fr_params *params, const uint64_t *seeds, const int32_t *spp,
                    float *const *out) {
    if (!b) return FR_EINVAL;
    b->err.clear();
    if (!params || !seeds || !spp || !out) return bfail(b, FR_EINVAL, "fr_batch_render: null argument");
    for (int i = 0; i < b->n; ++i) {
        const fr_ctx *c = b->ctx[i];
        const fr_params *p = &params[i];
        if (!out[i] || !p->lights || !p->spec || !p->pose || (c->n_id && !p->alpha) || (c->n_exp && !p->beta) ||
            (c->n_alb && !p->delta))
            return bfail(b, FR_EINVAL, "fr_batch_render: null argument of instance %d", i);
        if (spp[i] < 1 || spp[i] > 4096)
            return bfail(b, FR_EINVAL, "fr_batch_render: instance %d: spp %d out of [1, 4096]", i, spp[i]);
        if ((long long)c->W * c->H * spp[i] > (1ll << 31) - 1)
            return bfail(b, FR_EINVAL, "fr_batch_render: instance %d: W*H*spp too large", i);
        for (int k = 0; k < 6; ++k)
            if (!std::isfinite(p->pose[k]))
                return bfail(b, FR_EINVAL, "fr_batch_render: instance %d: non-finite pose[%d]", i, k);
        if (c->stream != b->stream)
            return bfail(b, FR_EINVAL, "fr_batch_render: instance %d is on another stream (fr_batch_set_stream)", i);
    }
    bool stale = b->spp.empty() || !std::equal(b->spp.begin(), b->spp.end(), spp);
    for (int i = 0; i < b->n && !stale; ++i) {   // a context's own render may have moved its scratch
        if (b->solo[i]) continue;
        const fr_ctx *c = b->ctx[i];
        const Inst &I = b->host[i];
        stale = c->hits != I.hits || c->vis != I.vis || c->samples != I.samples || c->sec_list != I.sec_list ||
                c->sh_queue != I.sh_queue || (uint32_t)c->sh_cap != I.sh_qcap;
    }
    if (stale) {
        int r = configure(b, spp);
        if (r) return r;
    }
    if (b->plan_dirty) {
        if (b->capturing) return bfail(b, FR_ESTATE, "fr_batch_render: launch plan changed during graph capture");
        int r = build_plan(b);
        if (r) return r;
    }
    for (int i = 0; i < b->n; ++i) {
        fr_ctx *c = b->ctx[i];
        const fr_params *p = &params[i];
        InstDyn &d = b->dyn[i];
        d = InstDyn{};
        d.seed = seeds[i]; d.spp = spp[i]; d.terms = (int)c->terms;
        rotation(p->pose, d.P.R);
        for (int k = 0; k < 3; ++k) d.P.t[k] = (double)p->pose[3 + k];
        drotation(p->pose, d.D.dR);
        d.alpha = p->alpha; d.beta = p->beta; d.delta = p->delta; d.lights = p->lights; d.spec = p->spec;
        d.img = out[i];
        if (b->solo[i]) continue;     // its own render sets its state
        // the context's own state, so that fr_backward / fr_aov on it follow this render
        c->last = *p;
        c->last_seed = seeds[i];
        c->last_spp = spp[i];
        c->last_cam_chunk = b->N[i];
        c->pose = d.P;
        c->drot = d.D;
    }
    const bool tm = (b->flags & FR_TIMING) && !b->capturing;
    if (tm) (void)hipEventRecord(b->ev[2 * bkNum], b->stream);
    put_dyn(b);
    seq_forward(b);
    for (int i = 0; i < b->n; ++i) {
        if (!b->solo[i]) continue;
        const int r = solo_call(b, i, [&](fr_ctx *c) { return render_call(c, &params[i], seeds[i], spp[i], out[i]); });
        if (r) return r;
    }
    if (tm) (void)hipEventRecord(b->ev[2 * bkNum + 1], b->stream);
    BHIPCK(b, hipGetLastError());
    for (int i = 0; i < b->n; ++i) {
        fr_ctx *c = b->ctx[i];
        if (b->solo[i]) { b->gen[i] = c->gen; continue; }
        c->records_valid = true;
        c->have_render = true;
        c->have_backward = false;
        b->gen[i] = ++c->gen;
    }
    b->have_render = true;
    b->have_backward = false;
    return FR_OK;
}

int fr_batch_backward(fr_batch *b, const float *const *dLdI, const fr_grads *grads) {
    if (!b) return FR_EINVAL;
    b->err.clear();
    if (!b->have_render) return bfail(b, FR_ESTATE, "fr_batch_backward: no prior fr_batch_render");
    if (!dLdI || !grads) return bfail(b, FR_EINVAL, "fr_batch_backward: null argument");
    for (int i = 0; i < b->n; ++i) {
        if (!dLdI[i]) return bfail(b, FR_EINVAL, "fr_batch_backward: null dL/dimage of instance %d", i);
        if (b->ctx[i]->gen != b->gen[i])
            return bfail(b, FR_ESTATE, "fr_batch_backward: instance %d was rendered on its own since", i);
    }
    for (int i = 0; i < b->n; ++i) {
        InstDyn &d = b->dyn[i];
        const fr_grads &g = grads[i];
        d.terms = (int)b->ctx[i]->terms;
        d.dLdI = dLdI[i];
        d.d_alpha = g.d_alpha; d.d_beta = g.d_beta; d.d_delta = g.d_delta; d.d_pose = g.d_pose;
        d.d_lights = g.d_lights; d.d_spec = g.d_spec; d.d_vertices = g.d_vertices; d.d_albedo = g.d_albedo;
        d.want_params = g.d_alpha || g.d_beta || g.d_delta || g.d_pose;
    }
    const bool tm = (b->flags & FR_TIMING) && !b->capturing;
    if (tm) (void)hipEventRecord(b->ev[2 * bkNum + 2], b->stream);
    put_dyn(b);
    seq_backward(b);
    for (int i = 0; i < b->n; ++i) {
        if (!b->solo[i]) continue;
        const int r = solo_call(b, i, [&](fr_ctx *c) { return backward_call(c, dLdI[i], &grads[i]); });
        if (r) return r;
    }
    if (tm) (void)hipEventRecord(b->ev[2 * bkNum + 3], b->stream);
    BHIPCK(b, hipGetLastError());
    for (fr_ctx *c : b->ctx) c->have_backward = true;
    b->have_backward = true;
    return FR_OK;
}

int fr_batch_timing(fr_batch *b, float *ms_kind, float *ms_render, float *ms_backward) {
    if (!b) return FR_EINVAL;
    b->err.clear();
    if (!(b->flags & FR_TIMING)) return bfail(b, FR_ESTATE, "fr_batch_timing: batch created without FR_TIMING");
    BHIPCK(b, hipStreamSynchronize(b->stream));
    float t;
    for (int k = 0; k < bkNum; ++k) {
        float v = 0.0f;
        if (b->timed[k] && hipEventElapsedTime(&t, b->ev[2 * k], b->ev[2 * k + 1]) == hipSuccess) v = t;
        if (ms_kind) ms_kind[k] = v;
    }
    if (ms_render) *ms_render = hipEventElapsedTime(&t, b->ev[2 * bkNum], b->ev[2 * bkNum + 1]) == hipSuccess ? t : 0.0f;
    if (ms_backward)
        *ms_backward = b->have_backward && hipEventElapsedTime(&t, b->ev[2 * bkNum + 2], b->ev[2 * bkNum + 3]) == hipSuccess
                           ? t : 0.0f;
    (void)hipGetLastError();
    return FR_OK;
}

// Autotuner: replays the last render and backward (same parameters, seeds,
// inputs and outputs) and chooses the launches by coordinate descent on the
// whole step's time: for each tunable kind in turn, each of its candidates
// with every other kind at its current choice, 'trials' replays each, the
// fastest (by its median) kept before the next kind.  Kinds interact through
// the placement of their tiles on the XCDs (a kind reads in its L2 what the
// kind before it wrote there), so a kind's own time alone can mislead.
// ms_best receives each kind's own time in the final choice.
static int replay_ms(fr_batch *b, int trials, float *ms) {
    std::vector<float> t(trials);
    for (int tr = 0; tr < trials; ++tr) {
        if (b->plan_dirty) { int rc = build_plan(b); if (rc) return rc; }
        BHIPCK(b, hipEventRecord(b->ev[2 * bkNum + 4], b->stream));
        seq_forward(b);
        seq_backward(b);
        BHIPCK(b, hipEventRecord(b->ev[2 * bkNum + 5], b->stream));
        BHIPCK(b, hipGetLastError());
        BHIPCK(b, hipStreamSynchronize(b->stream));
        BHIPCK(b, hipEventElapsedTime(&t[tr], b->ev[2 * bkNum + 4], b->ev[2 * bkNum + 5]));
    }
    std::sort(t.begin(), t.end());
    *ms = t[trials / 2];
    return FR_OK;
}

int fr_batch_tune(fr_batch *b, int32_t trials, float *ms_best) {
    if (!b) return FR_EINVAL;
    b->err.clear();
    if (!(b->flags & FR_TIMING)) return bfail(b, FR_ESTATE, "fr_batch_tune: batch created without FR_TIMING");
    if (!b->have_backward) return bfail(b, FR_ESTATE, "fr_batch_tune: needs a prior render and backward");
    if (b->capturing) return bfail(b, FR_ESTATE, "fr_batch_tune: graph capture in progress");
    if (trials < 1 || trials > 16) return bfail(b, FR_EINVAL, "fr_batch_tune: trials %d out of [1, 16]", trials);
    BHIPCK(b, hipStreamSynchronize(b->stream));
    float ms;
    int rc = replay_ms(b, 1, &ms);      // one untimed warm replay
    if (rc) return rc;
    for (int k = 0; k < bkNum; ++k) {
        if (!kind_tunable(k)) continue;
        std::vector<fr_launch> cand;
        const int nt = kind_tiled(k) ? 2 : 1;
        for (int t = 0; t < nt; ++t) {
            const int ts = kind_tiled(k) ? kTiles[t] : 0;
            cand.push_back(fr_launch{FR_LAUNCH_FLAT, ts});
            cand.push_back(fr_launch{FR_LAUNCH_XCD, ts});
        }
        fr_launch best = b->launch[k];
        float best_ms = INFINITY;
        for (const fr_launch &L : cand) {
            if (L.tile != b->launch[k].tile) b->plan_dirty = true;
            b->launch[k] = L;
            if ((rc = replay_ms(b, trials, &ms))) return rc;
            if (ms < best_ms) { best_ms = ms; best = L; }
        }
        if (best.tile != b->launch[k].tile) b->plan_dirty = true;
        b->launch[k] = best;
    }
    if ((rc = replay_ms(b, 1, &ms))) return rc;   // per-kind times of the choice
    for (int k = 0; k < bkNum; ++k) {
        float t = 0.0f;
        if (kind_tunable(k) && b->timed[k]) (void)hipEventElapsedTime(&t, b->ev[2 * k], b->ev[2 * k + 1]);
        if (ms_best) ms_best[k] = kind_tunable(k) ? t : 0.0f;
    }
    (void)hipGetLastError();
    return FR_OK;
}

int fr_batch_capture_begin(fr_batch *b) {
    if (!b) return FR_EINVAL;
    b->err.clear();
    if (b->capturing) return bfail(b, FR_ESTATE, "fr_batch_capture_begin: capture already in progress");
    if (!b->stream) return bfail(b, FR_ESTATE, "fr_batch_capture_begin: the null stream cannot be captured");
    if (b->spp.empty() || b->plan_dirty)
        return bfail(b, FR_ESTATE, "fr_batch_capture_begin: run the batch once before capturing it");
    BHIPCK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    b->capturing = true;
    return FR_OK;
}

int fr_batch_capture_end(fr_batch *b) {
    if (!b) return FR_EINVAL;
    b->err.clear();
    if (!b->capturing) return bfail(b, FR_ESTATE, "fr_batch_capture_end: no capture in progress");
    b->capturing = false;
    hipGraph_t g = nullptr;
    BHIPCK(b, hipStreamEndCapture(b->stream, &g));
    bool updated = false;
    if (b->exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        updated = hipGraphExecUpdate(b->exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        (void)hipGetLastError();
        if (!updated) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    }
    if (!b->exec) {
        hipError_t e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            b->exec = nullptr;
            return bfail(b, FR_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
    }
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph = g;
    return FR_OK;
}

int fr_batch_graph_launch(fr_batch *b) {
    if (!b) return FR_EINVAL;
    b->err.clear();
    if (!b->exec) return bfail(b, FR_ESTATE, "fr_batch_graph_launch: nothing captured");
    if (b->capturing) return bfail(b, FR_ESTATE, "fr_batch_graph_launch: capture in progress");
    BHIPCK(b, hipGraphLaunch(b->exec, b->stream));
    return FR_OK;
}

const char *fr_batch_last_error(const fr_batch *b) { return b ? b->err.c_str() : kNoCtx; }

void fr_batch_destroy(fr_batch *b) {
    if (!b) return;
    if (b->capturing) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(b->stream, &g);
        if (g) (void)hipGraphDestroy(g);
    }
    if (b->stream) (void)hipStreamSynchronize(b->stream); else (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->tab) (void)hipFree(b->tab);
    if (b->plan) (void)hipFree(b->plan);
    for (auto &e : b->ev) if (e) (void)hipEventDestroy(e);
    (void)hipGetLastError();
    delete b;
}

}  // extern "C"
