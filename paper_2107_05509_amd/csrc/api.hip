// C ABI of the handrt library (include/handrt.h): scene set-up on the host
// (topology tables, bounding-volume hierarchy topology, work lists) and the
// per-iteration launch sequences.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/handrt.h"
#include "kernels.hip"
#include "proposal.hip"
#include "dataterm.hip"
#include "bvh_build.h"

using namespace hr;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HR_EHIP, "%s: %s", what, hipGetErrorString(e));
    return HR_OK;
}

template <class T>
int dev_upload(T** dst, const T* src, size_t n)
{
    *dst = nullptr;
    if (n == 0) return HR_OK;
    hipError_t e = hipMalloc((void**)dst, sizeof(T) * n);
    if (e != hipSuccess) return fail(HR_EHIP, "hipMalloc(%zu): %s", sizeof(T) * n, hipGetErrorString(e));
    if (src) {
        e = hipMemcpy(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(HR_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
    }
    return HR_OK;
}

}  // namespace

// Scratch of hr_loss_noalloc (chunk partial sums, then the views' loss
// scales): a fixed array of the library, one copy per device, held until the
// process ends.  Host code reaches a device's copy only through the address
// hipGetSymbolAddress returns on that device (the symbol's name is a host
// stand-in, not a device address).
constexpr int kScratchFloats = 1 << 14;   // 64 KiB
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

// this device's copy of `scratch`, looked up once per device (with `dev` current)
int scratch_address(int dev, float** out)
{
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return fail(HR_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HR_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_dev[dev];
    return HR_OK;
}

}  // namespace

struct hr_scene {
    int device = 0;
    int n_hands = 0, n_views = 0;
    int V = 0, F = 0, J = 0, K = 0, E = 0;
    long long n_pixels = 0;
    hr_config cfg{};
    MeshDev mesh{};
    BvhDev bvh{};
    int bvh_depth = 0;
    std::vector<void*> allocs;
    ViewDev* views = nullptr;
    std::vector<ViewDev> views_host;
    TileShape ts{};
    int2* tiles = nullptr;        // wave tiles inside the per-view screen bounds
    uint64_t* hit_rec = nullptr;  // [tile_cap, rounds, 64] samples of the last render (random word, leaf slot)
    int* hit_iter = nullptr;      // iteration of those hits (-1: none)
    int4* view_rect = nullptr;    // [n_views] pixel rectangle of each view's tiles (screen-bounds pass)
    BinDev bins{};                // screen bins of the camera rays (built by the preparation launch)
    int bin_log2 = kBinLog2;      // bins of 2^bin_log2 pixels square
    bool layout_changed = false;  // hr_set_tiles since the last preparation
    int renderer = HR_RENDERER_RAY;
    int edge_div = 256;           // quantised silhouette length (1/256 px) per edge sample
    bool render_edges = false;    // hr_render also traces the edge samples (hr_set_render_edges)
    bool edges_valid = false;     // ... and has done so for the current preparation, at iteration edges_iter
    uint32_t edges_iter = 0;
    float* raster_image = nullptr;   // [P,3] hard rasterisation: image of a stand-alone backward's render
    long long bin_cap = 0;        // bins of all views at the smallest bin size
    int accel = HR_ACCEL_AUTO;
    long long tile_cap = 0;
    int* tile_count = nullptr;
    int render_blocks = 0;        // persistent grids of the ray-tracing kernels (hr_tune)
    int adjoint_blocks = 0;
    int max_blocks = 0;           // one block per 4 wave tiles of the full views
    int2* chunks = nullptr;
    int n_chunks = 0;
    int* view_chunk_off = nullptr;
    int* hand_view_off = nullptr;
    int* hand_views = nullptr;
    int max_views_per_hand = 0;
    float* normals = nullptr;
    Tri* tris = nullptr;
    // joint prior (hr_set_joint_prior): caller-owned target joints, weight, threshold
    const float* prior_target = nullptr;
    float prior_lambda = 0.0f, prior_gamma = 1.0f;
    Node* nodes = nullptr;
    float* gacc = nullptr;        // [views,V,3] float64 vertex gradient slots of each view (edge term),
                                  // zeroed as 6 floats per vertex
    float* gface = nullptr;       // [hands,F,18] triangle corner slots (interior term)
    EdgeSample* samples = nullptr;   // traced edge samples (first part of the boundary term)
    long long sample_cap = 0;
    int skin_blocks = 0;
    float* loss_partial = nullptr;
    float* view_scale = nullptr;
    EdgeRec* edge_rec = nullptr;
    unsigned long long* edge_cdf = nullptr;
    unsigned long long* edge_total = nullptr;
    long long* edge_budget = nullptr;
    long long* edge_prefix = nullptr;
    int* setup_done = nullptr;
    size_t smem_prepare = 0;
    float* geom_gr = nullptr;     // [hands,V,3] geometry backward: raw-normal gradients
    float* geom_gpos = nullptr;   // [hands,V,3] slot gradients
    float* geom_part = nullptr;   // [hands,kSkinPart] skinning sums (zero between launches)
    int* geom_count = nullptr;    // [hands] finished blocks (reset by the last)
    float* joint_state = nullptr; // [hands, joint state] of hr_iterate's skinning, for its backward
    float* bvh_cost = nullptr;    // [hands] traversal cost of the last refitted hierarchy
    int* hand_counter = nullptr;  // [1] hands finished in the geometry backward (reset by the last)
    int geom_blocks = 0;
    unsigned long long* counts = nullptr;   // [3][6] work counters (render, interior adjoint, edges)
    int n_cu = 0;                 // compute units of the scene's device
    // full data term (hr_data_term_set, hr_edge_map, hr_loss_full)
    bool dt_alloc = false;
    DataTermDev dt{};
    // learned edge-sampling proposal (hr_proposal_*)
    bool prop_alloc = false;
    int prop_kind = HR_PROPOSAL_LENGTH;
    PropDev prop{};
    float* fit_z = nullptr;
    // side stream of hr_iterate: the proposal pass runs beside the loss, its
    // training beside the geometry backward and the parameter step
    hipStream_t side = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};   // hr_iterate: after the ray-tracing backward; end of training
    bool counting = false;
    // per-kernel timing (profiling aid)
    bool timing = false;
    struct TimedLaunch { const char* name; hipEvent_t a, b; };
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;

    template <class T>
    int upload(T** dst, const T* src, size_t n)
    {
        int rc = dev_upload(dst, src, n);
        if (*dst) allocs.push_back((void*)*dst);
        return rc;
    }
};

struct hr_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int n_iters = 0;
};

// Copy one hand's hierarchy topology to the device (synchronous).  Internal
// nodes are renumbered by height, the root first (index 0, where traversal
// starts) and the nodes of each height contiguous: the refit walks a height
// as one index range.  With it go the vertex ids of each leaf slot's triangle.
static int upload_hierarchy(hr_scene* s, int h, const HostBvh& hb, const int* faces)
{
    BvhDev& b = s->bvh;
    const int n = (int)hb.child.size() / 2;
    const int nl = (int)hb.level_off.size() - 1;
    if (hb.depth + 1 > kMaxStack || nl + 1 > b.level_stride)
        return fail(HR_EUNSUPPORTED, "hierarchy too deep (%d levels)", hb.depth);
    if (n > b.node_stride) return fail(HR_EUNSUPPORTED, "hierarchy too large (%d nodes)", n);
    if ((int)hb.order.size() != n || hb.level_off[nl] != n) return fail(HR_EINVAL, "hierarchy: bad level order");
    std::vector<int> renum(n), child(2 * (size_t)n);
    for (int q = 0; q < n; ++q) renum[hb.order[q]] = n - 1 - q;
    if (renum[0] != 0) return fail(HR_EINVAL, "hierarchy: the root is not the highest node");
    for (int old = 0; old < n; ++old)
        for (int c = 0; c < 2; ++c) {
            const int code = hb.child[2 * (size_t)old + c];
            child[2 * (size_t)renum[old] + c] = code >= 0 ? renum[code] : code;
        }
    std::vector<int> order(n), sv((size_t)s->F * 3);
    for (int q = 0; q < n; ++q) order[q] = n - 1 - q;
    for (int i = 0; i < s->F; ++i)
        for (int k = 0; k < 3; ++k) sv[3 * (size_t)i + k] = faces[3 * (size_t)hb.perm[i] + k];
    hipError_t e = hipMemcpy((int*)b.child + (size_t)h * b.node_stride * 2, child.data(),
                             sizeof(int) * child.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy((int*)b.perm + (size_t)h * s->F, hb.perm.data(), sizeof(int) * hb.perm.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy((int*)b.order + (size_t)h * b.node_stride, order.data(), sizeof(int) * order.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy((int*)b.slot_verts + (size_t)h * s->F * 3, sv.data(), sizeof(int) * sv.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy((int*)b.level_off + (size_t)h * b.level_stride, hb.level_off.data(),
                      sizeof(int) * hb.level_off.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy((int*)b.n_levels + h, &nl, sizeof(int), hipMemcpyHostToDevice);
    // the triangles' face and vertex ids (the refit writes their corners)
    std::vector<Tri> tri(s->F);
    for (int i = 0; i < s->F; ++i) {
        Tri& t = tri[i];
        std::fill(t.v, t.v + 9, 0.0f);
        t.face = hb.perm[i];
        t.i0 = sv[3 * (size_t)i]; t.i1 = sv[3 * (size_t)i + 1]; t.i2 = sv[3 * (size_t)i + 2];
        t.pad[0] = t.pad[1] = t.pad[2] = 0;
    }
    if (e == hipSuccess)
        e = hipMemcpy(s->tris + (size_t)h * s->F, tri.data(), sizeof(Tri) * tri.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(HR_EHIP, "hierarchy upload: %s", hipGetErrorString(e));
    return HR_OK;
}

// Launch a kernel; with timing enabled, bracket it by events on its stream.
template <class... KArgs, class... Args>
static int launch(hr_scene* s, const char* name, void (*kern)(KArgs...), dim3 grid, dim3 block, size_t smem,
                  hipStream_t st, Args... args)
{
    hr_scene::TimedLaunch tl{name, nullptr, nullptr};
    if (s->timing) {
        for (hipEvent_t* ev : {&tl.a, &tl.b}) {
            if (!s->event_pool.empty()) { *ev = s->event_pool.back(); s->event_pool.pop_back(); }
            else if (hipEventCreate(ev) != hipSuccess) return fail(HR_EHIP, "%s: hipEventCreate failed", name);
        }
        (void)hipEventRecord(tl.a, st);
    }
    hipLaunchKernelGGL(kern, grid, block, smem, st, args...);
    int rc = check_launch(name);
    if (s->timing) {
        (void)hipEventRecord(tl.b, st);
        s->timed.push_back(tl);
    }
    return rc;
}

extern "C" {

const char* hr_last_error(void) { return g_err.c_str(); }

void hr_scene_destroy(hr_scene* s)
{
    if (!s) return;
    for (auto& t : s->timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (void* p : s->allocs) (void)hipFree(p);
    for (hipEvent_t e : s->ev)
        if (e) (void)hipEventDestroy(e);
    if (s->side) (void)hipStreamDestroy(s->side);
    delete s;
}

int64_t hr_num_pixels(const hr_scene* s) { return s ? s->n_pixels : -1; }

// First bin and bins per row of every view for the scene's bin size (host copy).
static void layout_bins(hr_scene* s)
{
    const int lb = s->bin_log2;
    long long n = 0;
    for (ViewDev& d : s->views_host) {
        d.bin0 = (int)n;
        d.nbx = (d.W + (1 << lb) - 1) >> lb;
        n += (long long)d.nbx * ((d.H + (1 << lb) - 1) >> lb);
    }
}

int hr_scene_create(hr_scene** out, const hr_mesh_desc* m, int32_t n_hands, const hr_camera* cams,
                    int32_t n_views, const hr_config* cfg)
{
    if (!out || !m || !cams || !cfg) return fail(HR_EINVAL, "hr_scene_create: null argument");
    *out = nullptr;
    if (n_hands < 1 || n_views < 1) return fail(HR_EINVAL, "hr_scene_create: need >= 1 hand and view");
    if (!m->v_template || !m->shapedirs || !m->j_regressor || !m->weights || !m->parents || !m->faces ||
        !m->uv || !m->edges || !m->edge_faces)
        return fail(HR_EINVAL, "hr_scene_create: null mesh array");
    const int V = m->n_verts, F = m->n_faces, J = m->n_joints, K = m->n_shape, E = m->n_edges;
    if (V < 3 || F < 1 || J < 1 || K < 0 || E < 3) return fail(HR_EINVAL, "hr_scene_create: bad mesh sizes");
    if (V > 4096 || F > 8192 || J > kMaxJoints || K > 16)
        return fail(HR_EUNSUPPORTED, "hr_scene_create: mesh too large (V<=4096, F<=8192, J<=32, K<=16)");
    if (cfg->spp < 1 || cfg->spp > 256) return fail(HR_EUNSUPPORTED, "hr_scene_create: spp must be 1..256");
    if (cfg->tex_h < 1 || cfg->tex_w < 1) return fail(HR_EINVAL, "hr_scene_create: bad texture size");
    if (!(cfg->edge_delta > 0.0f)) return fail(HR_EINVAL, "hr_scene_create: edge_delta must be > 0");
    for (int f = 0; f < 3 * F; ++f)
        if (m->faces[f] < 0 || m->faces[f] >= V) return fail(HR_EINVAL, "hr_scene_create: face index out of range");
    for (int e = 0; e < E; ++e) {
        if (m->edges[2 * e] < 0 || m->edges[2 * e] >= V || m->edges[2 * e + 1] < 0 || m->edges[2 * e + 1] >= V)
            return fail(HR_EINVAL, "hr_scene_create: edge vertex out of range");
        if (m->edge_faces[2 * e] < 0 || m->edge_faces[2 * e] >= F || m->edge_faces[2 * e + 1] >= F)
            return fail(HR_EINVAL, "hr_scene_create: edge face out of range");
    }
    for (int j = 0; j < J; ++j)
        if (m->parents[j] >= j || (j > 0 && m->parents[j] < 0) || (j == 0 && m->parents[0] >= 0))
            return fail(HR_EINVAL, "hr_scene_create: parents must satisfy parents[0] < 0 <= parents[j] < j");
    for (int v = 0; v < n_views; ++v) {
        const hr_camera& c = cams[v];
        if (c.hand < 0 || c.hand >= n_hands) return fail(HR_EINVAL, "hr_scene_create: camera %d: bad hand", v);
        if (c.W < 1 || c.H < 1) return fail(HR_EINVAL, "hr_scene_create: camera %d: bad size", v);
        if (c.W > 4096 || c.H > 4096) return fail(HR_EUNSUPPORTED, "hr_scene_create: camera %d larger than 4096", v);
        if (!(c.fx > 0.0f) || !(c.fy > 0.0f)) return fail(HR_EINVAL, "hr_scene_create: camera %d: bad focal", v);
    }

    hr_scene* s = new hr_scene();
    s->n_hands = n_hands;
    s->n_views = n_views;
    s->V = V; s->F = F; s->J = J; s->K = K; s->E = E;
    s->cfg = *cfg;
    (void)hipGetDevice(&s->device);
    int rc = HR_OK;
#define TRY(x) do { rc = (x); if (rc != HR_OK) { hr_scene_destroy(s); return rc; } } while (0)
    {
        float* sp;   // hr_loss_noalloc's scratch on this device (looked up here, once per device)
        TRY(scratch_address(s->device, &sp));
    }
    // mesh tables
    MeshDev& md = s->mesh;
    md.V = V; md.F = F; md.J = J; md.K = K; md.E = E;
    {
        float* p;
        // per-vertex tables vertex-minor ([..][V]): a wave's 64 vertices read
        // one contiguous run per entry
        {
            std::vector<float> tt(3 * (size_t)V), st(3 * (size_t)V * std::max(K, 1), 0.0f);
            for (int v = 0; v < V; ++v)
                for (int c = 0; c < 3; ++c) {
                    tt[(size_t)c * V + v] = m->v_template[3 * (size_t)v + c];
                    for (int k = 0; k < K; ++k)
                        st[((size_t)k * 3 + c) * V + v] = m->shapedirs[(3 * (size_t)v + c) * K + k];
                }
            TRY(s->upload(&p, tt.data(), tt.size())); md.v_template = p;
            TRY(s->upload(&p, st.data(), st.size())); md.shapedirs = p;
        }
        TRY(s->upload(&p, m->j_regressor, (size_t)J * V)); md.j_regressor = p;
        TRY(s->upload(&p, m->weights, (size_t)V * J)); md.weights = p;
        TRY(s->upload(&p, m->uv, 2 * (size_t)V)); md.uv = p;
        int* q;
        TRY(s->upload(&q, m->parents, (size_t)J)); md.parents = q;
        TRY(s->upload(&q, m->faces, 3 * (size_t)F)); md.faces = q;
        TRY(s->upload(&q, m->edges, 2 * (size_t)E)); md.edges = q;
        TRY(s->upload(&q, m->edge_faces, 2 * (size_t)E)); md.edge_faces = q;
        // per edge: its vertices, then the vertices of its faces in face
        // order (-1 for a missing second face): one table read per edge
        std::vector<int> et((size_t)E * 8, -1);
        for (int e = 0; e < E; ++e) {
            et[8 * (size_t)e] = m->edges[2 * e];
            et[8 * (size_t)e + 1] = m->edges[2 * e + 1];
            for (int k = 0; k < 2; ++k) {
                const int f = m->edge_faces[2 * e + k];
                if (f < 0) continue;
                for (int c = 0; c < 3; ++c) et[8 * (size_t)e + 2 + 3 * k + c] = m->faces[3 * f + c];
            }
        }
        TRY(s->upload(&q, et.data(), et.size())); md.edge_verts = reinterpret_cast<const int4*>(q);
        std::vector<int> off(V + 1, 0), cnt(V, 0), flat(3 * F);
        for (int i = 0; i < 3 * F; ++i) off[m->faces[i] + 1]++;
        for (int v = 0; v < V; ++v) off[v + 1] += off[v];
        for (int f = 0; f < F; ++f)
            for (int k = 0; k < 3; ++k) {
                int v = m->faces[3 * f + k];
                flat[off[v] + cnt[v]++] = f;
            }
        TRY(s->upload(&q, off.data(), off.size())); md.vf_off = q;
        TRY(s->upload(&q, flat.data(), flat.size())); md.vf_faces = q;
        // the same lists as (vertex triple, face), kVfSlots per vertex, padded
        // with (v, v, v, 0): a degenerate face adds nothing to the normal backward
        std::vector<int> vc(4 * (size_t)V * kVfSlots, 0);
        for (int v = 0; v < V; ++v)
            for (int k = 0; k < kVfSlots; ++k) {
                int* d = &vc[4 * ((size_t)k * V + v)];
                if (off[v] + k < off[v + 1]) {
                    const int f = flat[off[v] + k];
                    for (int c = 0; c < 3; ++c) d[c] = m->faces[3 * f + c];
                    d[3] = f;
                } else {
                    d[0] = d[1] = d[2] = v;
                    d[3] = 0;
                }
            }
        TRY(s->upload(&q, vc.data(), vc.size())); md.vf_corner = reinterpret_cast<const int4*>(q);
        // regressor applied to the template and to the shape directions (float64 sums)
        std::vector<float> jt(3 * (size_t)J), jsd(3 * (size_t)J * std::max(K, 1), 0.0f);
        std::vector<double> jt64(jt.size()), jsd64(jsd.size(), 0.0);
        for (int j = 0; j < J; ++j)
            for (int c = 0; c < 3; ++c) {
                double a = 0.0;
                for (int v = 0; v < V; ++v) a += (double)m->j_regressor[(size_t)j * V + v] * m->v_template[3 * v + c];
                jt[3 * j + c] = (float)a;
                jt64[3 * j + c] = a;
                for (int k = 0; k < K; ++k) {
                    double b = 0.0;
                    for (int v = 0; v < V; ++v)
                        b += (double)m->j_regressor[(size_t)j * V + v] * m->shapedirs[((size_t)3 * v + c) * K + k];
                    jsd[(3 * (size_t)j + c) * K + k] = (float)b;
                    jsd64[(3 * (size_t)j + c) * K + k] = b;
                }
            }
        float* pf;
        TRY(s->upload(&pf, jt.data(), jt.size())); md.jt = pf;
        TRY(s->upload(&pf, jsd.data(), jsd.size())); md.js = pf;
        double* pd;
        TRY(s->upload(&pd, jt64.data(), jt64.size())); md.jt64 = pd;
        TRY(s->upload(&pd, jsd64.data(), jsd64.size())); md.js64 = pd;
        std::vector<int> depth(J, 0);
        int maxd = 0;
        for (int j = 0; j < J; ++j) {
            depth[j] = m->parents[j] < 0 ? 0 : depth[m->parents[j]] + 1;
            maxd = std::max(maxd, depth[j]);
        }
        TRY(s->upload(&q, depth.data(), depth.size())); md.jdepth = q;
        md.max_depth = maxd;
        // non-zero skinning weights per vertex, padded to the largest count
        int infl = 1;
        for (int v = 0; v < V; ++v) {
            int c = 0;
            for (int j = 0; j < J; ++j) c += m->weights[(size_t)v * J + j] != 0.0f;
            infl = std::max(infl, c);
        }
        std::vector<int> widx((size_t)V * infl, 0);
        std::vector<float> wval((size_t)V * infl, 0.0f);
        for (int v = 0; v < V; ++v) {
            int c = 0;
            for (int j = 0; j < J; ++j) {
                const float w = m->weights[(size_t)v * J + j];
                if (w != 0.0f) { widx[(size_t)c * V + v] = j; wval[(size_t)c * V + v] = w; ++c; }
            }
        }
        if (infl > kMaxInfl) {
            hr_scene_destroy(s);
            return fail(HR_EUNSUPPORTED, "hr_scene_create: a vertex has %d skinning weights (at most %d)", infl,
                        kMaxInfl);
        }
        md.infl = infl;
        TRY(s->upload(&q, widx.data(), widx.size())); md.widx = q;
        TRY(s->upload(&pf, wval.data(), wval.size())); md.wval = pf;
    }
    // hierarchy topology: from the rest pose until hr_build_hierarchy is called
    {
        BvhDev& b = s->bvh;
        b.node_stride = std::max(F - 1, 1);
        b.level_stride = kMaxStack + 2;
        int* q;
        TRY(s->upload<int>(&q, nullptr, (size_t)n_hands)); b.n_levels = q;
        TRY(s->upload<int>(&q, nullptr, (size_t)n_hands * b.node_stride * 2)); b.child = q;
        TRY(s->upload<int>(&q, nullptr, (size_t)n_hands * F)); b.perm = q;
        TRY(s->upload<int>(&q, nullptr, (size_t)n_hands * b.node_stride)); b.order = q;
        TRY(s->upload<int>(&q, nullptr, (size_t)n_hands * b.level_stride)); b.level_off = q;
        TRY(s->upload<int>(&q, nullptr, (size_t)n_hands * F * 3)); b.slot_verts = q;
        TRY(s->upload<Tri>(&s->tris, nullptr, (size_t)n_hands * F));
        HostBvh hb = build_bvh(m->v_template, m->faces, F, kLeafMax);
        for (int h = 0; h < n_hands; ++h) TRY(upload_hierarchy(s, h, hb, m->faces));
    }
    // views, work lists
    {
        // wave tile shape: all samples of a pixel in one wave
        TileShape& ts = s->ts;
        int spp_r = 1, lg = 0;
        while (spp_r < cfg->spp && spp_r < 64) { spp_r <<= 1; ++lg; }
        ts.spp_log2 = lg;
        const int ppw_log2 = 6 - lg;
        ts.tw_log2 = (ppw_log2 + 1) / 2;
        ts.th_log2 = ppw_log2 - ts.tw_log2;
        ts.rounds = (cfg->spp + 63) / 64;
        std::vector<int2> chunks;
        std::vector<int> vco(1, 0);
        long long pix = 0, bin_cap = 0;
        for (int v = 0; v < n_views; ++v) {
            const hr_camera& c = cams[v];
            ViewDev d;
            memcpy(d.R, c.R, sizeof(d.R));
            memcpy(d.o, c.o, sizeof(d.o));
            d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
            d.W = c.W; d.H = c.H; d.hand = c.hand;
            d.sid = cfg->view_base + (uint32_t)v;
            // bins: room for the smallest bin size; tiles: for the shape with the most tiles
            bin_cap += ((c.W + (1 << kMinBinLog2) - 1) >> kMinBinLog2) * ((c.H + (1 << kMinBinLog2) - 1) >> kMinBinLog2);
            d.pix0 = pix;
            long long tmax = 0;
            for (int tw = 0; tw <= ppw_log2; ++tw)
                tmax = std::max(tmax, (long long)((c.W + (1 << tw) - 1) >> tw) *
                                          ((c.H + (1 << (ppw_log2 - tw)) - 1) >> (ppw_log2 - tw)));
            s->tile_cap += tmax;
            const long long np = (long long)c.W * c.H;
            for (long long p0 = 0; p0 < np; p0 += kLossChunk) chunks.push_back(make_int2(v, (int)p0));
            vco.push_back((int)chunks.size());
            pix += np;
            s->views_host.push_back(d);
        }
        s->n_pixels = pix;
        s->bin_cap = bin_cap;
        layout_bins(s);
        s->n_chunks = (int)chunks.size();
        s->max_blocks = (int)std::max<long long>(1, std::min<long long>(kMaxTraceBlocks, (s->tile_cap + 3) / 4));
        s->render_blocks = s->adjoint_blocks = std::min(2048, s->max_blocks);
        std::vector<int> hvo(n_hands + 1, 0), hv;
        for (int h = 0; h < n_hands; ++h) {
            for (int v = 0; v < n_views; ++v)
                if (cams[v].hand == h) hv.push_back(v);
            hvo[h + 1] = (int)hv.size();
            s->max_views_per_hand = std::max(s->max_views_per_hand, hvo[h + 1] - hvo[h]);
        }
        TRY(s->upload(&s->views, s->views_host.data(), s->views_host.size()));
        TRY(s->upload(&s->chunks, chunks.data(), chunks.size()));
        TRY(s->upload(&s->view_chunk_off, vco.data(), vco.size()));
        TRY(s->upload(&s->hand_view_off, hvo.data(), hvo.size()));
        TRY(s->upload(&s->hand_views, hv.data(), hv.size()));
    }
    // per-iteration state
    TRY(s->upload<int2>(&s->tiles, nullptr, (size_t)s->tile_cap));
    TRY(s->upload<uint64_t>(&s->hit_rec, nullptr, (size_t)s->tile_cap * s->ts.rounds * 64));
    TRY(s->upload<int>(&s->hit_iter, nullptr, 1));
    TRY(s->upload<int4>(&s->view_rect, nullptr, (size_t)n_views));
    {   // screen bins: entries for each triangle in up to 16 bins per view on average
        BinDev& bd = s->bins;
        bd.cap = 16 * F;
        bd.log2 = s->bin_log2;
        TRY(s->upload<int>(&bd.count, nullptr, (size_t)s->bin_cap));
        TRY(s->upload<int>(&bd.off, nullptr, (size_t)s->bin_cap));
        TRY(s->upload<uint16_t>(&bd.entries, nullptr, (size_t)n_views * bd.cap));
        TRY(s->upload<float4>(&bd.box, nullptr, (size_t)n_views * F));
        TRY(s->upload<int>(&bd.binned, nullptr, (size_t)n_views));
        if (hipMemset(bd.binned, 0, sizeof(int) * n_views) != hipSuccess) {
            hr_scene_destroy(s);
            return fail(HR_EHIP, "scene init: memset");
        }
    }

    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            hr_scene_destroy(s);
            return fail(HR_EHIP, "scene init: device attributes");
        }
    }
    if (hipMemset(s->hit_iter, 0xFF, sizeof(int)) != hipSuccess) {
        hr_scene_destroy(s);
        return fail(HR_EHIP, "scene init: memset");
    }
    TRY(s->upload<int>(&s->tile_count, nullptr, 4));
    TRY(s->upload<float>(&s->normals, nullptr, (size_t)n_hands * V * 3));
    TRY(s->upload<Node>(&s->nodes, nullptr, (size_t)n_hands * s->bvh.node_stride));
    TRY(s->upload<float>(&s->gacc, nullptr, (size_t)n_views * V * 6));
    TRY(s->upload<float>(&s->gface, nullptr, (size_t)n_hands * F * 18));
    {   // stored edge samples: generous for hand silhouettes; samples beyond are traced in place
        long long cap = 65536;
        for (int v = 0; v < n_views; ++v) cap += 8ll * (cams[v].W + cams[v].H);
        s->sample_cap = cap;
        TRY(s->upload<EdgeSample>(&s->samples, nullptr, (size_t)cap));
    }
    s->skin_blocks = (V + 127) / 128;
    s->geom_blocks = (V + 63) / 64;
    TRY(s->upload<float>(&s->geom_gr, nullptr, (size_t)n_hands * V * 3));
    TRY(s->upload<float>(&s->geom_gpos, nullptr, (size_t)n_hands * V * 3));
    TRY(s->upload<float>(&s->geom_part, nullptr, (size_t)n_hands * kSkinPart));
    if (hipMemset(s->geom_part, 0, sizeof(float) * n_hands * kSkinPart) != hipSuccess) {
        hr_scene_destroy(s);
        return fail(HR_EHIP, "scene init: memset");
    }
    TRY(s->upload<int>(&s->geom_count, nullptr, (size_t)n_hands));
    TRY(s->upload<float>(&s->joint_state, nullptr, (size_t)n_hands * kJointStateFloats));
    {
        const std::vector<float> zero((size_t)n_hands, 0.0f);   // 0 until the first refit
        TRY(s->upload(&s->bvh_cost, zero.data(), zero.size()));
    }
    TRY(s->upload<int>(&s->hand_counter, nullptr, 1));
    TRY(s->upload<int>(&s->setup_done, nullptr, 1));
    if (hipMemset(s->hand_counter, 0, sizeof(int)) != hipSuccess ||
        hipMemset(s->setup_done, 0, sizeof(int)) != hipSuccess) {
        hr_scene_destroy(s);
        return fail(HR_EHIP, "scene init: memset");
    }
    if (hipMemset(s->geom_count, 0, sizeof(int) * n_hands) != hipSuccess) {
        hr_scene_destroy(s);
        return fail(HR_EHIP, "scene init: memset");
    }
    TRY(s->upload<float>(&s->loss_partial, nullptr, 2 * (size_t)s->n_chunks));
    TRY(s->upload<float>(&s->view_scale, nullptr, n_views));
    TRY(s->upload<EdgeRec>(&s->edge_rec, nullptr, (size_t)n_views * E));
    TRY(s->upload<unsigned long long>(&s->edge_cdf, nullptr, (size_t)n_views * E));
    TRY(s->upload<unsigned long long>(&s->edge_total, nullptr, n_views));
    TRY(s->upload<long long>(&s->edge_budget, nullptr, n_views));
    TRY(s->upload<long long>(&s->edge_prefix, nullptr, (size_t)n_views + 1));
    TRY(s->upload<unsigned long long>(&s->counts, nullptr, kCounts));
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, (hipStream_t)0, s->counts, kCounts);
    if (hipDeviceSynchronize() != hipSuccess) { hr_scene_destroy(s); return fail(HR_EHIP, "scene init failed"); }
    if (hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess) {
        hr_scene_destroy(s);
        return fail(HR_EHIP, "scene init: stream");
    }
    for (hipEvent_t& ev : s->ev)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            hr_scene_destroy(s);
            return fail(HR_EHIP, "scene init: event");
        }
#undef TRY
    // refit: vertices, node bounds, slot bounds, child codes and the leaf
    // slots' vertex ids; normals: vertices and face normals
    s->smem_prepare = sizeof(float) * (3 * V + 6 * s->bvh.node_stride + 6 * F) +
                      sizeof(int) * (2 * s->bvh.node_stride + 3 * F + s->bvh.level_stride);
    s->smem_prepare = std::max(s->smem_prepare, sizeof(float) * (3 * V + 3 * F));
    // silhouette-table blocks: scan buffer, edge table, vertices, edge weights
    s->smem_prepare = std::max(s->smem_prepare, sizeof(unsigned long long) * 16 + sizeof(int) * 8 * E +
                                                    sizeof(float) * 3 * V + sizeof(uint32_t) * E);
    // bin blocks: projected vertices, two counters per (bin, depth band) cell
    s->smem_prepare = std::max(s->smem_prepare, sizeof(float) * 3 * V + sizeof(int) * 2 * kMaxBinCells);
    if (hipFuncSetAttribute((const void*)k_prepare, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)s->smem_prepare) != hipSuccess) {
        hr_scene_destroy(s);
        return fail(HR_EUNSUPPORTED, "hr_scene_create: mesh needs more LDS than a workgroup has");
    }
    *out = s;
    return HR_OK;
}

int hr_skin(hr_scene* s, const float* params, float* verts, float* joints, void* stream)
{
    if (!s || !params || !verts) return fail(HR_EINVAL, "hr_skin: null argument");
    hipStream_t st = (hipStream_t)stream;
    return launch(s, "k_skin", k_skin, dim3(s->skin_blocks, s->n_hands), dim3(128), 0, st, s->mesh, params, verts,
                  joints, (int*)nullptr, (float*)nullptr);
}

int hr_build_hierarchy(hr_scene* s, const float* verts, void* stream)
{
    if (!s || !verts) return fail(HR_EINVAL, "hr_build_hierarchy: null argument");
    hipStream_t st = (hipStream_t)stream;
    std::vector<float> hv((size_t)s->n_hands * s->V * 3);
    std::vector<int> faces((size_t)s->F * 3);
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(hv.data(), verts, sizeof(float) * hv.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(faces.data(), s->mesh.faces, sizeof(int) * faces.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_build_hierarchy: %s", hipGetErrorString(e));
    for (size_t i = 0; i < hv.size(); ++i)
        if (!std::isfinite(hv[i])) return fail(HR_EINVAL, "hr_build_hierarchy: non-finite vertex");
    for (int h = 0; h < s->n_hands; ++h) {
        HostBvh hb = build_bvh(hv.data() + (size_t)h * s->V * 3, faces.data(), s->F, kLeafMax);
        int rc = upload_hierarchy(s, h, hb, faces.data());
        if (rc) return rc;
    }
    // the stored samples of an earlier render name leaf slots of the old
    // topology: a backward reusing them prepares and traces again
    s->layout_changed = true;
    s->edges_valid = false;
    if (hipMemset(s->hit_iter, 0xFF, sizeof(int)) != hipSuccess)
        return fail(HR_EHIP, "hr_build_hierarchy: memset");
    return HR_OK;
}

int hr_hierarchy_cost(hr_scene* s, float* cost_host)
{
    if (!s || !cost_host) return fail(HR_EINVAL, "hr_hierarchy_cost: null argument");
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(cost_host, s->bvh_cost, sizeof(float) * s->n_hands, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_hierarchy_cost: %s", hipGetErrorString(e));
    return HR_OK;
}

static EdgeArgs edge_args(hr_scene* s, const float* verts, const float* albedo, const float* background,
                          const float* dimage, uint32_t iter, const int* iter_dev);

// Everything the render and the backward need from the vertices, one
// launch: refit, silhouette tables, wave tiles and (with_scale) the views'
// loss scales from the mask.  reset_tiles: zero the tile count first (the
// iteration folds that into its skinning launch instead).
static int prepare(hr_scene* s, const float* verts, hipStream_t st, bool reset_tiles = true, bool with_scale = false,
                   const uint8_t* mask = nullptr)
{
    s->layout_changed = false;
    s->edges_valid = false;   // a new geometry: the traced edge samples are stale
    if (reset_tiles) {
        const int rc = launch(s, "k_set_i32", k_set_i32, dim3(1), dim3(64), 0, st, s->tile_count, 1, 0);
        if (rc) return rc;
    }
    PrepArgs a;
    a.m = s->mesh; a.b = s->bvh; a.verts = verts; a.normals = s->normals; a.tris = s->tris; a.nodes = s->nodes;
    a.e = edge_args(s, verts, nullptr, nullptr, nullptr, 0, nullptr);
    a.views = s->views; a.ts = s->ts; a.tiles = s->tiles; a.tile_count = s->tile_count; a.view_rect = s->view_rect;
    a.mask = mask; a.view_scale = s->view_scale; a.setup_done = s->setup_done;
    a.bins = s->bins;
    a.with_bins = s->accel == HR_ACCEL_AUTO ? 1 : 0;
    a.bvh_cost = s->bvh_cost;
    a.n_hands = s->n_hands; a.n_views = s->n_views; a.with_setup = 1; a.with_scale = with_scale;
    const dim3 grid(2 * s->n_hands + (3 + (with_scale ? 1 : 0)) * s->n_views);
    return launch(s, "k_prepare", k_prepare, grid, dim3(512), s->smem_prepare, st, a);
}

static Shading shading_of(const hr_config& c)
{
    Shading S;
    S.ka = c.ka; S.kd = c.kd;
    S.l[0] = c.light[0]; S.l[1] = c.light[1]; S.l[2] = c.light[2];
    return S;
}

// `dimage` (with target, mask): the L1 loss gradient is written with the
// image, scaled by the view_scale a preceding prepare (with_scale) left.
// n_edge > 0: the render blocks also trace the edge samples, each its share
// after its tiles (the weights and budget prefix are built beforehand:
// edge_trace_impl, trace false).
static int render_impl(hr_scene* s, const float* verts, const float* albedo, const float* background, uint32_t iter,
                       const int* iter_dev, float* image, int32_t* hit_face, hipStream_t st, bool prepared = false,
                       float* const* clear = nullptr, const long long* clear_n = nullptr,
                       const float* target = nullptr, const uint8_t* mask = nullptr, float* dimage = nullptr,
                       int n_edge = 0)
{
    int rc = prepared ? HR_OK : prepare(s, verts, st);
    if (rc) return rc;
    const long long P = s->n_pixels;
    if (hit_face) {
        rc = launch(s, "k_fill_i32", k_fill_i32, dim3((unsigned)std::min<long long>(4096, (P * s->cfg.spp + 255) / 256)),
                    dim3(256), 0, st, (int*)hit_face, P * s->cfg.spp, -1);
        if (rc) return rc;
    }
    RenderArgs a;
    a.tiles = s->tiles; a.tile_count = s->tile_count; a.ts = s->ts; a.views = s->views;
    a.nodes = s->nodes; a.tris = s->tris; a.normals = s->normals; a.uv = s->mesh.uv;
    a.albedo = albedo; a.background = background; a.image = image; a.hit_face = hit_face;
    a.hit_rec = s->hit_rec; a.hit_iter = s->hit_iter;
    a.view_rect = s->view_rect; a.n_views = s->n_views;
    a.dimage = dimage; a.target = target; a.mask = mask; a.view_scale = s->view_scale;
    for (int k = 0; k < 3; ++k) {
        a.clear[k] = clear ? clear[k] : nullptr;
        a.clear_n[k] = clear ? clear_n[k] : 0;
    }
    a.n_nodes = s->bvh.node_stride; a.n_faces = s->F; a.n_verts = s->V;
    a.tex_h = s->cfg.tex_h; a.tex_w = s->cfg.tex_w; a.spp = s->cfg.spp;
    a.iter = iter; a.iter_dev = iter_dev; a.seed = s->cfg.seed; a.shading = shading_of(s->cfg);
    a.counts = s->counts;
    a.bins = s->bins;
    const bool raster = s->renderer == HR_RENDERER_RASTER;   // hard rasterisation: its own kernel instantiation
    const EdgeArgs e = edge_args(s, verts, albedo, background, nullptr, iter, iter_dev);
    const dim3 grid(s->render_blocks);
    const int with_edges = n_edge > 0 && !raster ? 1 : 0;
    if (raster) {
        if (s->counting) return launch(s, "k_render", k_render<true, true>, grid, dim3(kThreads), 0, st, a, e, 0);
        return launch(s, "k_render", k_render<false, true>, grid, dim3(kThreads), 0, st, a, e, 0);
    }
    // few tiles: the tiles of all views at most one wave per SIMD (4 per CU)
    if (s->tile_cap <= 4LL * s->n_cu && grid.x >= 2) {
        if (s->counting)
            return launch(s, "k_render", k_render_few<true>, grid, dim3(kThreads), 0, st, a, e, with_edges);
        return launch(s, "k_render", k_render_few<false>, grid, dim3(kThreads), 0, st, a, e, with_edges);
    }
    if (s->counting) return launch(s, "k_render", k_render<true, false>, grid, dim3(kThreads), 0, st, a, e, with_edges);
    return launch(s, "k_render", k_render<false, false>, grid, dim3(kThreads), 0, st, a, e, with_edges);
}

// Edge samples, first part: silhouette tables (unless done), learned sampling
// weights, budget prefix, tracing of every stored sample.

static int edge_trace_impl(hr_scene* s, const float* verts, const float* albedo, const float* background,
                           uint32_t iter, const int* iter_dev, hipStream_t st, bool trace = true)
{
    EdgeArgs e = edge_args(s, verts, albedo, background, nullptr, iter, iter_dev);
    int rc = HR_OK;
    if (!rc && s->prop_kind == HR_PROPOSAL_LEARNED)
        rc = launch(s, "k_proposal", k_proposal, dim3(s->n_views, s->prop.split), dim3(256), 0, st, e, s->prop);
    // the preparation launch wrote the prefix of the length budgets; the
    // learned proposal's budgets need their own
    if (!rc && s->prop_kind == HR_PROPOSAL_LEARNED)
        rc = launch(s, "k_edge_prefix", k_edge_prefix, dim3(1), dim3(256), 0, st, (const long long*)s->edge_budget,
                    s->n_views, s->edge_prefix);
    if (rc || !trace) return rc;
    if (s->counting) return launch(s, "k_edge_trace", k_edge_trace<true>, dim3(kEdgeBlocks), dim3(kThreads), 0, st, e);
    return launch(s, "k_edge_trace", k_edge_trace<false>, dim3(kEdgeBlocks), dim3(kThreads), 0, st, e);
}

int hr_render(hr_scene* s, const float* verts, const float* albedo, const float* background, uint32_t iter,
              float* image, int32_t* hit_face, void* stream)
{
    if (!s || !verts || !albedo || !background || !image) return fail(HR_EINVAL, "hr_render: null argument");
    hipStream_t st = (hipStream_t)stream;
    if (!s->render_edges || s->renderer == HR_RENDERER_RASTER)
        return render_impl(s, verts, albedo, background, iter, nullptr, image, hit_face, st);
    // the edge samples' side rays traced by the render launch, for a
    // following hr_backward with HR_REUSE_GEOMETRY at the same iteration
    int rc = prepare(s, verts, st);
    if (!rc) rc = edge_trace_impl(s, verts, albedo, background, iter, nullptr, st, false);
    if (!rc)
        rc = render_impl(s, verts, albedo, background, iter, nullptr, image, hit_face, st, true, nullptr, nullptr,
                         nullptr, nullptr, nullptr, kEdgeBlocks);
    if (!rc) {
        s->edges_valid = true;
        s->edges_iter = iter;
    }
    return rc;
}

int hr_set_render_edges(hr_scene* s, int32_t enable)
{
    if (!s) return fail(HR_EINVAL, "hr_set_render_edges: null scene");
    s->render_edges = enable != 0;
    return HR_OK;
}

static EdgeArgs edge_args(hr_scene* s, const float* verts, const float* albedo, const float* background,
                          const float* dimage, uint32_t iter, const int* iter_dev)
{
    EdgeArgs a;
    a.m = s->mesh; a.views = s->views; a.verts = verts;
    a.rec = s->edge_rec; a.cdf = s->edge_cdf; a.total = s->edge_total; a.budget = s->edge_budget;
    a.prefix = s->edge_prefix; a.n_views = s->n_views; a.budget_div = s->edge_div;
    a.nodes = s->nodes; a.tris = s->tris; a.normals = s->normals; a.uv = s->mesh.uv;
    a.albedo = albedo; a.background = background; a.dimage = dimage; a.gacc = s->gacc;
    a.stat_a = nullptr; a.stat_dc = nullptr;
    a.samples = s->samples; a.sample_cap = s->sample_cap; a.few_waves = s->n_cu;
    a.counts = s->counts + 12;
    a.n_nodes = s->bvh.node_stride; a.tex_h = s->cfg.tex_h; a.tex_w = s->cfg.tex_w;
    a.delta = s->cfg.edge_delta; a.iter = iter; a.iter_dev = iter_dev; a.seed = s->cfg.seed;
    a.shading = shading_of(s->cfg);
    return a;
}

int hr_set_counting(hr_scene* s, int32_t enable)
{
    if (!s) return fail(HR_EINVAL, "hr_set_counting: null scene");
    s->counting = enable != 0;
    return HR_OK;
}

int hr_read_counts(hr_scene* s, uint64_t* counts_host, void* stream)
{
    if (!s || !counts_host) return fail(HR_EINVAL, "hr_read_counts: null argument");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(counts_host, s->counts, kCounts * sizeof(uint64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_read_counts: %s", hipGetErrorString(e));
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, s->counts, kCounts);
    return check_launch("hr_read_counts");
}

int hr_timing_enable(hr_scene* s, int32_t enable)
{
    if (!s) return fail(HR_EINVAL, "hr_timing_enable: null scene");
    s->timing = enable != 0;
    return HR_OK;
}

int hr_timing_read(hr_scene* s, char* names, double* ms, int64_t* count, int32_t max_n, int32_t* n_out, void* stream)
{
    if (!s || !names || !ms || !count || !n_out || max_n < 1) return fail(HR_EINVAL, "hr_timing_read: bad argument");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_timing_read: %s", hipGetErrorString(e));
    std::vector<std::string> keys;
    std::vector<double> tot;
    std::vector<int64_t> cnt;
    for (auto& t : s->timed) {
        (void)hipEventSynchronize(t.b);
        float x = 0.0f;
        (void)hipEventElapsedTime(&x, t.a, t.b);
        size_t k = 0;
        while (k < keys.size() && keys[k] != t.name) ++k;
        if (k == keys.size()) { keys.push_back(t.name); tot.push_back(0.0); cnt.push_back(0); }
        tot[k] += x;
        cnt[k] += 1;
        s->event_pool.push_back(t.a);
        s->event_pool.push_back(t.b);
    }
    s->timed.clear();
    int n = (int)std::min<size_t>(keys.size(), (size_t)max_n);
    for (int i = 0; i < n; ++i) {
        memset(names + 32 * i, 0, 32);
        strncpy(names + 32 * i, keys[i].c_str(), 31);
        ms[i] = tot[i];
        count[i] = cnt[i];
    }
    *n_out = n;
    return HR_OK;
}

static int loss_impl(hr_scene* s, const float* image, const float* target, const uint8_t* mask, float* loss,
                     float* dimage, hipStream_t st)
{
    LossArgs a;
    a.chunks = s->chunks; a.views = s->views; a.image = image; a.target = target; a.mask = mask;
    a.partial = s->loss_partial; a.view_chunk_off = s->view_chunk_off; a.hand_view_off = s->hand_view_off;
    a.hand_views = s->hand_views; a.view_scale = s->view_scale; a.loss = loss; a.dimage = dimage;
    a.n_hands = s->n_hands;
    int rc = launch(s, "k_loss_partial", k_loss_partial, dim3(s->n_chunks), dim3(256), 0, st, a);
    if (rc) return rc;
    rc = launch(s, "k_loss_final", k_loss_final, dim3(s->n_hands), dim3(256), 0, st, a);
    if (rc) return rc;
    return launch(s, "k_loss_grad", k_loss_grad, dim3(s->n_chunks), dim3(256), 0, st, a);
}


int hr_loss(hr_scene* s, const float* image, const float* target, const uint8_t* mask, float* loss, float* dimage,
            void* stream)
{
    if (!s || !image || !target || !loss || !dimage) return fail(HR_EINVAL, "hr_loss: null argument");
    return loss_impl(s, image, target, mask, loss, dimage, (hipStream_t)stream);
}

int hr_loss_noalloc(hr_scene* s, const float* image, const float* target, const uint8_t* mask, float* loss,
                    float* dimage, void* stream)
{
    if (!s || !image || !target || !loss || !dimage) return fail(HR_EINVAL, "hr_loss_noalloc: null argument");
    const long long need = 2LL * s->n_chunks + s->n_views;
    if (need > kScratchFloats)
        return fail(HR_EUNSUPPORTED,
                    "hr_loss_noalloc: the scene needs %lld scratch floats (%d chunks of %d pixels, %d views), "
                    "the fixed array holds %d", need, s->n_chunks, kLossChunk, s->n_views, kScratchFloats);
    float* sp = nullptr;
    const int rc = scratch_address(s->device, &sp);   // set at scene creation: a table read
    if (rc) return rc;
    const hipStream_t st = (hipStream_t)stream;
    LossArgs a;
    a.chunks = s->chunks; a.views = s->views; a.image = image; a.target = target; a.mask = mask;
    a.partial = sp; a.view_chunk_off = s->view_chunk_off; a.hand_view_off = s->hand_view_off;
    a.hand_views = s->hand_views; a.view_scale = sp + 2 * (size_t)s->n_chunks; a.loss = loss; a.dimage = dimage;
    a.n_hands = s->n_hands;
    // every value is written before it is read (partials, then scales): nothing to clear
    hipLaunchKernelGGL(k_loss_partial, dim3(s->n_chunks), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_loss_final, dim3(s->n_hands), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_loss_grad, dim3(s->n_chunks), dim3(256), 0, st, a);
    return check_launch("hr_loss_noalloc");
}

static int fill(hr_scene* s, float* p, long long n, float v, hipStream_t st)
{
    if (n <= 0) return HR_OK;
    long long blocks = std::min<long long>((n + 255) / 256, 4096);
    return launch(s, "k_fill", k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

static AdamArgs adam_args(hr_scene* s, float* params, float* albedo, const float* grad_params,
                          const float* grad_albedo, float* m_params, float* v_params, float* m_albedo, float* v_albedo,
                          int32_t t, const int* iter_dev, const hr_adam_config* cfg)
{
    AdamArgs a;
    a.params = params; a.albedo = albedo; a.grad_params = grad_params; a.grad_albedo = grad_albedo;
    a.m_params = m_params; a.v_params = v_params; a.m_albedo = m_albedo; a.v_albedo = v_albedo;
    a.n_albedo = (long long)s->n_hands * s->cfg.tex_h * s->cfg.tex_w * 3;
    a.n_hands = s->n_hands;
    a.lr[0] = cfg->lr_pose_root; a.lr[1] = cfg->lr_pose; a.lr[2] = cfg->lr_shape;
    a.lr[3] = cfg->lr_rot; a.lr[4] = cfg->lr_trans; a.lr[5] = cfg->lr_albedo;
    a.beta1 = cfg->beta1; a.beta2 = cfg->beta2; a.eps = cfg->eps;
    a.bc1 = (float)(1.0 - std::pow((double)cfg->beta1, (double)t));
    a.bc2 = (float)(1.0 - std::pow((double)cfg->beta2, (double)t));
    a.iter_dev = iter_dev;
    return a;
}

// the Adam kernel over a's parameters (a.n_hands of them, 0: colour map only)
// and colour map, four colour-map entries per thread and step
static int adam_launch(hr_scene* s, const AdamArgs& a, hipStream_t st)
{
    const long long n = 64ll * a.n_hands + a.n_albedo / 4;
    const unsigned blocks = (unsigned)std::max<long long>(1, std::min<long long>(2048, (n + 255) / 256));
    return launch(s, "k_adam", k_adam, dim3(blocks), dim3(256), 0, st, a);
}

static int backward_impl(hr_scene* s, const float* params, const float* verts, const float* albedo,
                         const float* background, const float* dimage, uint32_t iter, const int* iter_dev,
                         uint32_t flags, float* grad_params, float* grad_albedo, float* grad_verts,
                         float* grad_normals, hipStream_t st, bool edges_traced = false,
                         hipEvent_t after_trace = nullptr, bool cleared = false, const AdamArgs* adam = nullptr,
                         const LossArgs* loss_value = nullptr, const float* js_saved = nullptr,
                         int* iter_advance = nullptr)
{
    int rc;
    if (s->renderer == HR_RENDERER_RASTER) {
        // hard rasterisation: no visibility (edge) term; the covering triangles
        // come from a render of these vertices (into the scene's scratch image
        // unless the caller's render of the same geometry is reused)
        flags &= ~HR_GRAD_EDGES;
        if (!(flags & HR_REUSE_GEOMETRY) || s->layout_changed) {
            rc = render_impl(s, verts, albedo, background, iter, iter_dev, s->raster_image, nullptr, st);
            if (rc) return rc;
            flags |= HR_REUSE_GEOMETRY;
        }
    }
    // reuse needs a preparation with the current work layout
    if (!(flags & HR_REUSE_GEOMETRY) || s->layout_changed) {
        rc = prepare(s, verts, st);
        if (rc) return rc;
    }
    if (!cleared) {
        const long long nalb = (long long)s->n_hands * s->cfg.tex_h * s->cfg.tex_w * 3;
        rc = fill(s, grad_albedo, nalb, 0.0f, st);
        if (!rc) rc = fill(s, s->gacc, (long long)s->n_views * s->V * 6, 0.0f, st);
        if (!rc) rc = fill(s, s->gface, (long long)s->n_hands * s->F * 18, 0.0f, st);
        if (rc) return rc;
    }
    EdgeArgs e = edge_args(s, verts, albedo, background, dimage, iter, iter_dev);
    int n_edge = 0, n_adj = 0;
    if (flags & HR_GRAD_EDGES) {
        // first part of the edge samples (tracing; learned sampling weights
        // replace the length weights of the CDF), unless the caller ran it
        if (!edges_traced) {
            rc = edge_trace_impl(s, verts, albedo, background, iter, iter_dev, st);
            if (rc) return rc;
        }
        if (s->prop_kind == HR_PROPOSAL_LEARNED) {   // per-edge records for training
            e.stat_a = s->prop.stat_a;
            e.stat_dc = s->prop.stat_dc;
        }
        n_edge = kEdgeBlocks;
    }
    AdjointArgs a;
    a.tiles = s->tiles; a.tile_count = s->tile_count; a.ts = s->ts; a.views = s->views;
    a.faces = s->mesh.faces;
    a.nodes = s->nodes; a.tris = s->tris; a.normals = s->normals; a.uv = s->mesh.uv;
    a.albedo = albedo; a.dimage = dimage; a.grad_albedo = grad_albedo; a.gface = s->gface;
    // the render's hits are valid for the geometry it prepared
    a.hit_rec = (flags & HR_REUSE_GEOMETRY) ? s->hit_rec : nullptr;
    a.hit_iter = s->hit_iter;
    a.n_nodes = s->bvh.node_stride; a.n_faces = s->F; a.n_verts = s->V;
    a.tex_h = s->cfg.tex_h; a.tex_w = s->cfg.tex_w; a.spp = s->cfg.spp;
    a.iter = iter; a.iter_dev = iter_dev; a.seed = s->cfg.seed; a.shading = shading_of(s->cfg);
    a.counts = s->counts + 6;
    if (flags & HR_GRAD_INTERIOR) n_adj = s->adjoint_blocks;
    // loss_value: the loss's chunk partials ride along (summed per hand by
    // the geometry backward)
    const int n_loss = loss_value ? s->n_chunks : 0;
    const LossArgs l = loss_value ? *loss_value : LossArgs{};
    if (n_edge + n_adj + n_loss > 0) {
        const dim3 grid(n_edge + n_adj + n_loss);
        if (s->counting)
            rc = launch(s, "k_backward_trace", k_backward_trace<true>, grid, dim3(kThreads), 0, st, a, e, n_edge, l,
                        n_loss);
        else
            rc = launch(s, "k_backward_trace", k_backward_trace<false>, grid, dim3(kThreads), 0, st, a, e, n_edge, l,
                        n_loss);
        if (rc) return rc;
    }
    if (after_trace && hipEventRecord(after_trace, st) != hipSuccess) return fail(HR_EHIP, "hr_backward: event");
    GeomBwdArgs g;
    g.m = s->mesh; g.params = params; g.verts = verts; g.gacc = s->gacc; g.gface = s->gface;
    g.hand_view_off = s->hand_view_off; g.hand_views = s->hand_views;
    g.grad_verts = grad_verts; g.grad_normals = grad_normals; g.grad_params = grad_params;
    // adam: the colour map's step (its gradient is final now) in blocks of
    // the first launch, the parameters' step at the end of each hand's
    // second launch; iter_advance: the counter advances after both
    g.adam_params = adam != nullptr;
    if (adam) g.adam = *adam;
    g.with_loss = loss_value != nullptr;
    if (loss_value) g.loss = *loss_value;
    g.gr = s->geom_gr; g.gpos = s->geom_gpos; g.part = s->geom_part; g.counter = s->geom_count;
    g.js_saved = js_saved;
    g.n_hands = s->n_hands;
    g.p1_blocks = (s->V + 255) / 256;
    g.iter_advance = iter_advance;
    g.hand_counter = s->hand_counter;
    const bool prior = !(flags & HR_SKIP_PRIOR);
    g.prior_target = prior ? s->prior_target : nullptr;
    g.prior_lambda = s->prior_lambda; g.prior_gamma = s->prior_gamma;
    // per hand one more block sums the loss value
    const long long n4 = (long long)s->n_hands * s->cfg.tex_h * s->cfg.tex_w * 3 / 4;
    const int n_adam = adam ? (int)std::min<long long>(1024, std::max<long long>(1, (n4 + 255) / 256)) : 0;
    rc = launch(s, "k_geom_p1", k_geom_p1, dim3(s->n_hands * (g.p1_blocks + 1) + n_adam), dim3(256), 0, st, g);
    if (!rc) rc = launch(s, "k_geom_p2", k_geom_p2, dim3(s->geom_blocks, s->n_hands), dim3(64), 0, st, g);
    return rc;
}

int hr_set_joint_prior(hr_scene* s, const float* target_joints, float lambda, float gamma)
{
    if (!s) return fail(HR_EINVAL, "hr_set_joint_prior: null scene");
    if (!(lambda >= 0.0f) || !std::isfinite(lambda) || !(gamma > 0.0f) || !std::isfinite(gamma))
        return fail(HR_EINVAL, "hr_set_joint_prior: need lambda >= 0 and gamma > 0 (finite)");
    const bool on = target_joints != nullptr && lambda > 0.0f;
    s->prior_target = on ? target_joints : nullptr;
    s->prior_lambda = on ? lambda : 0.0f;
    s->prior_gamma = gamma;
    return HR_OK;
}

int hr_face_visibility(hr_scene* s, const int32_t* hit_face, int32_t* visible, void* stream)
{
    if (!s || !hit_face || !visible) return fail(HR_EINVAL, "hr_face_visibility: null argument");
    const hipStream_t st = (hipStream_t)stream;
    const long long n = (long long)s->n_views * s->F;
    int rc = launch(s, "k_fill_i32", k_fill_i32, dim3((unsigned)std::min<long long>(1024, (n + 255) / 256)), dim3(256),
                    0, st, (int*)visible, n, 0);
    if (rc) return rc;
    const size_t smem = sizeof(unsigned int) * (size_t)((s->F + 31) / 32);
    if (smem > (size_t)kCoverLdsBytes) return fail(HR_EUNSUPPORTED, "hr_face_visibility: too many faces");
    return launch(s, "k_face_visibility", k_face_visibility, dim3(64, s->n_views), dim3(256), smem, st, s->views,
                  (const int*)hit_face, s->cfg.spp, s->F, (int*)visible);
}

int hr_camera_order(hr_scene* s, const int32_t* visible, int32_t* order, int32_t* covered, void* stream)
{
    if (!s || !visible || !order || !covered) return fail(HR_EINVAL, "hr_camera_order: null argument");
    const size_t nwords = (size_t)(s->F + 31) / 32, nwp = (nwords + 3) & ~(size_t)3, nv = (size_t)s->max_views_per_hand;
    const size_t smem = sizeof(unsigned int) * (nv * nwp + nwp + nv);
    if (smem > (size_t)kCoverLdsBytes)
        return fail(HR_EUNSUPPORTED, "hr_camera_order: the views' face bitmaps (%zu B) exceed %d B of LDS", smem,
                    kCoverLdsBytes);
    return launch(s, "k_camera_order", k_camera_order, dim3(s->n_hands), dim3(1024), smem, (hipStream_t)stream,
                  (const int*)visible, s->hand_view_off, s->hand_views, s->F, (int*)order, (int*)covered);
}

int hr_backward(hr_scene* s, const float* params, const float* verts, const float* albedo, const float* background,
                const float* dimage, uint32_t iter, uint32_t flags, float* grad_params, float* grad_albedo,
                float* grad_verts, float* grad_normals, void* stream)
{
    if (!s || !params || !verts || !albedo || !background || !dimage || !grad_params || !grad_albedo)
        return fail(HR_EINVAL, "hr_backward: null argument");
    if (flags & ~(HR_GRAD_ALL | HR_REUSE_GEOMETRY | HR_SKIP_PRIOR)) return fail(HR_EINVAL, "hr_backward: unknown flags");
    // edge samples traced by the last hr_render (hr_set_render_edges) of this geometry and iteration
    const bool traced = (flags & HR_REUSE_GEOMETRY) && s->edges_valid && s->edges_iter == iter && !s->layout_changed;
    return backward_impl(s, params, verts, albedo, background, dimage, iter, nullptr, flags, grad_params, grad_albedo,
                         grad_verts, grad_normals, (hipStream_t)stream, traced);
}

static int step_impl(hr_scene* s, float* params, float* albedo, const float* grad_params, const float* grad_albedo,
                     float* m_params, float* v_params, float* m_albedo, float* v_albedo, int32_t t, const int* iter_dev,
                     const hr_adam_config* cfg, hipStream_t st)
{
    return adam_launch(s, adam_args(s, params, albedo, grad_params, grad_albedo, m_params, v_params, m_albedo,
                                    v_albedo, t, iter_dev, cfg), st);
}

int hr_step(hr_scene* s, float* params, float* albedo, const float* grad_params, const float* grad_albedo,
            float* m_params, float* v_params, float* m_albedo, float* v_albedo, int32_t t, const hr_adam_config* cfg,
            void* stream)
{
    if (!s || !params || !albedo || !grad_params || !grad_albedo || !m_params || !v_params || !m_albedo ||
        !v_albedo || !cfg)
        return fail(HR_EINVAL, "hr_step: null argument");
    if (t < 1) return fail(HR_EINVAL, "hr_step: t must be >= 1");
    return step_impl(s, params, albedo, grad_params, grad_albedo, m_params, v_params, m_albedo, v_albedo, t, nullptr,
                     cfg, (hipStream_t)stream);
}

static int check_state(const hr_state* q, const char* who)
{
    if (!q) return fail(HR_EINVAL, "%s: null state", who);
    if (!q->params || !q->albedo || !q->m_params || !q->v_params || !q->m_albedo || !q->v_albedo ||
        !q->background || !q->target || !q->verts || !q->image || !q->dimage || !q->loss || !q->grad_params ||
        !q->grad_albedo || !q->iter)
        return fail(HR_EINVAL, "%s: null state buffer (only mask may be null)", who);
    return HR_OK;
}

// Training step of the learned proposal on the statistics of the last
// backward pass (no-op unless the proposal is learned and trainable).
static int proposal_train_impl(hr_scene* s, hipStream_t st)
{
    if (s->prop_kind != HR_PROPOSAL_LEARNED || s->prop.z_override || !(s->prop.lr > 0.0f)) return HR_OK;
    const int items = s->n_views * s->prop.split;
    int rc = launch(s, "k_proposal_train", k_proposal_train, dim3(std::min(items, 256)), dim3(256), 0, st,
                    (const EdgeRec*)s->edge_rec, s->E, s->n_views, s->prop);
    const long long rows = (long long)s->n_views * s->E;
    if (!rc)
        rc = launch(s, "k_proposal_ema", k_proposal_ema, dim3((unsigned)std::min<long long>(2048, (rows + 255) / 256)),
                    dim3(256), 0, st, s->prop, rows);
    return rc;
}

// One refinement iteration with the iteration index in device memory.
static int iterate_impl(hr_scene* s, const hr_state* q, const hr_adam_config* cfg, uint32_t flags, hipStream_t st)
{
    const int* it = q->iter;
    const bool raster = s->renderer == HR_RENDERER_RASTER;
    const bool learned = (flags & HR_GRAD_EDGES) && !raster && s->prop_kind == HR_PROPOSAL_LEARNED;
    const bool train = learned && !s->prop.z_override && s->prop.lr > 0.0f;
    auto join = [&](hipEvent_t ev) -> int {
        if (hipEventRecord(ev, s->side) != hipSuccess || hipStreamWaitEvent(st, ev, 0) != hipSuccess)
            return fail(HR_EHIP, "hr_iterate: join");
        return HR_OK;
    };
    // one stream: skinning (emptying the tile list), one preparation launch
    // (refit, silhouette tables, tiles, loss scales), the learned weights and
    // budget prefix, the render with the edge samples traced by its blocks and
    // the loss gradient written with the image, the ray-tracing backward with
    // the loss partial sums beside it, the geometry backward with the loss
    // values and both Adam steps; training of a learned proposal on the side
    // stream beside the geometry backward
    const bool edges = (flags & HR_GRAD_EDGES) != 0 && !raster;   // hard rasterisation has no edge term
    int rc = launch(s, "k_skin", k_skin, dim3(s->skin_blocks, s->n_hands), dim3(128), 0, st, s->mesh,
                    (const float*)q->params, q->verts, (float*)nullptr, s->tile_count, s->joint_state);
    if (!rc) rc = prepare(s, q->verts, st, false, true, q->mask);
    if (!rc && edges) rc = edge_trace_impl(s, q->verts, q->albedo, q->background, 0, it, st, false);
    float* const clr[3] = {q->grad_albedo, s->gacc, s->gface};
    const long long clr_n[3] = {(long long)s->n_hands * s->cfg.tex_h * s->cfg.tex_w * 3, (long long)s->n_views * s->V * 6,
                                (long long)s->n_hands * s->F * 18};
    if (!rc)
        rc = render_impl(s, q->verts, q->albedo, q->background, 0, it, q->image, nullptr, st, true, clr, clr_n,
                         q->target, q->mask, q->dimage, edges ? kEdgeBlocks : 0);
    LossArgs lv;
    lv.chunks = s->chunks; lv.views = s->views; lv.image = q->image; lv.target = q->target; lv.mask = q->mask;
    lv.partial = s->loss_partial; lv.view_chunk_off = s->view_chunk_off; lv.hand_view_off = s->hand_view_off;
    lv.hand_views = s->hand_views; lv.view_scale = nullptr; lv.loss = q->loss; lv.dimage = nullptr;
    lv.n_hands = s->n_hands;
    const AdamArgs adam = adam_args(s, q->params, q->albedo, q->grad_params, q->grad_albedo, q->m_params,
                                    q->v_params, q->m_albedo, q->v_albedo, 1, it, cfg);
    if (!rc)
        rc = backward_impl(s, q->params, q->verts, q->albedo, q->background, q->dimage, 0, it,
                           (flags & HR_GRAD_ALL) | HR_REUSE_GEOMETRY, q->grad_params, q->grad_albedo, nullptr,
                           nullptr, st, edges, train ? s->ev[0] : nullptr, true, &adam, &lv, s->joint_state,
                           train ? nullptr : q->iter);
    if (!rc && train && hipStreamWaitEvent(s->side, s->ev[0], 0) != hipSuccess) rc = fail(HR_EHIP, "hr_iterate: fork");
    if (!rc && train) rc = proposal_train_impl(s, s->side);
    if (!rc && train) rc = join(s->ev[1]);
    // with training the side stream still reads the counter: advance after the join
    if (!rc && train) rc = launch(s, "k_advance", k_advance, dim3(1), dim3(64), 0, st, q->iter);
    return rc;
}

int hr_iterate(hr_scene* s, const hr_state* state, const hr_adam_config* cfg, uint32_t flags, void* stream)
{
    if (!s || !cfg) return fail(HR_EINVAL, "hr_iterate: null argument");
    int rc = check_state(state, "hr_iterate");
    if (rc) return rc;
    if (flags & ~HR_GRAD_ALL) return fail(HR_EINVAL, "hr_iterate: unknown flags");
    return iterate_impl(s, state, cfg, flags, (hipStream_t)stream);
}

int hr_graph_create(hr_graph** out, hr_scene* s, const hr_state* state, const hr_adam_config* cfg, uint32_t flags,
                    int32_t n_iters)
{
    if (!out || !s || !cfg) return fail(HR_EINVAL, "hr_graph_create: null argument");
    *out = nullptr;
    int rc = check_state(state, "hr_graph_create");
    if (rc) return rc;
    if (flags & ~HR_GRAD_ALL) return fail(HR_EINVAL, "hr_graph_create: unknown flags");
    if (n_iters < 1 || n_iters > 1024) return fail(HR_EINVAL, "hr_graph_create: n_iters must be 1..1024");
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_graph_create: %s", hipGetErrorString(e));
    const bool timing = s->timing;
    s->timing = false;    // no event nodes in the graph
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) rc = fail(HR_EHIP, "hr_graph_create: begin capture: %s", hipGetErrorString(e));
    for (int i = 0; i < n_iters && !rc; ++i) rc = iterate_impl(s, state, cfg, flags, cs);
    if (e == hipSuccess) {
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (!rc && e2 != hipSuccess) rc = fail(HR_EHIP, "hr_graph_create: end capture: %s", hipGetErrorString(e2));
    }
    s->timing = timing;
    (void)hipStreamDestroy(cs);
    hipGraphExec_t x = nullptr;
    if (!rc) {
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = fail(HR_EHIP, "hr_graph_create: instantiate: %s", hipGetErrorString(e));
    }
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    hr_graph* h = new hr_graph();
    h->graph = g;
    h->exec = x;
    h->n_iters = n_iters;
    *out = h;
    return HR_OK;
}

int hr_graph_launch(hr_graph* g, void* stream)
{
    if (!g) return fail(HR_EINVAL, "hr_graph_launch: null graph");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_graph_launch: %s", hipGetErrorString(e));
    return HR_OK;
}

void hr_graph_destroy(hr_graph* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

int hr_set_grid(hr_scene* s, int32_t render_blocks, int32_t adjoint_blocks)
{
    if (!s) return fail(HR_EINVAL, "hr_set_grid: null scene");
    if (render_blocks < 0 || adjoint_blocks < 0) return fail(HR_EINVAL, "hr_set_grid: negative block count");
    if (render_blocks) s->render_blocks = std::min(render_blocks, s->max_blocks);
    if (adjoint_blocks) s->adjoint_blocks = std::min(adjoint_blocks, s->max_blocks);
    return HR_OK;
}

int hr_set_accel(hr_scene* s, int32_t mode)
{
    if (!s) return fail(HR_EINVAL, "hr_set_accel: null scene");
    if (mode != HR_ACCEL_AUTO && mode != HR_ACCEL_HIERARCHY) return fail(HR_EINVAL, "hr_set_accel: unknown mode %d", mode);
    s->accel = mode;
    return HR_OK;
}

// Wave-tile shape and screen-bin size.  Neither changes which samples are
// drawn or how a pixel's samples are summed, so images are bit-identical for
// every choice; the render's stored samples (kept by tile) are dropped.
static int set_tiles(hr_scene* s, int tw_log2, int bin_log2)
{
    const int ppw = s->ts.tw_log2 + s->ts.th_log2;   // pixels per wave, log2
    const int th_log2 = ppw - tw_log2;
    if (tw_log2 < 0 || th_log2 < 0 || bin_log2 < kMinBinLog2 || bin_log2 > kMaxBinLog2 || tw_log2 > bin_log2 ||
        th_log2 > bin_log2)
        return fail(HR_EINVAL, "hr_set_tiles: tile 2^%d x 2^%d pixels in bins of 2^%d pixels is not available "
                    "(tile sides 2^a x 2^b with a + b = %d, bins 2^%d .. 2^%d, a tile inside one bin)",
                    tw_log2, th_log2, bin_log2, ppw, kMinBinLog2, kMaxBinLog2);
    if (tw_log2 == s->ts.tw_log2 && bin_log2 == s->bin_log2) return HR_OK;
    // work already enqueued reads the views' bin layout and the stored samples
    if (hipDeviceSynchronize() != hipSuccess) return fail(HR_EHIP, "hr_set_tiles: synchronize");
    s->ts.tw_log2 = tw_log2;
    s->ts.th_log2 = th_log2;
    s->bin_log2 = bin_log2;
    s->bins.log2 = bin_log2;
    s->layout_changed = true;
    layout_bins(s);
    if (hipMemcpy(s->views, s->views_host.data(), sizeof(ViewDev) * s->views_host.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(s->hit_iter, 0xFF, sizeof(int)) != hipSuccess)
        return fail(HR_EHIP, "hr_set_tiles: upload");
    return HR_OK;
}

int hr_set_edge_budget(hr_scene* s, int32_t units_per_sample)
{
    if (!s) return fail(HR_EINVAL, "hr_set_edge_budget: null scene");
    if (units_per_sample < 1 || units_per_sample > (1 << 20))
        return fail(HR_EINVAL, "hr_set_edge_budget: %d outside 1 .. 2^20", units_per_sample);
    s->edge_div = units_per_sample;
    return HR_OK;
}

int hr_set_renderer(hr_scene* s, int32_t mode)
{
    if (!s) return fail(HR_EINVAL, "hr_set_renderer: null scene");
    if (mode != HR_RENDERER_RAY && mode != HR_RENDERER_RASTER) return fail(HR_EINVAL, "hr_set_renderer: unknown mode %d", mode);
    if (mode == HR_RENDERER_RASTER && s->cfg.spp != 1)
        return fail(HR_EUNSUPPORTED, "hr_set_renderer: hard rasterisation takes one sample per pixel (spp %d)", s->cfg.spp);
    if (mode == s->renderer) return HR_OK;
    if (hipDeviceSynchronize() != hipSuccess) return fail(HR_EHIP, "hr_set_renderer: synchronize");
    if (mode == HR_RENDERER_RASTER && !s->raster_image) {
        const int rc = s->upload<float>(&s->raster_image, nullptr, (size_t)s->n_pixels * 3);
        if (rc) return rc;
    }
    s->renderer = mode;
    // the stored samples belong to the other renderer
    if (hipMemset(s->hit_iter, 0xFF, sizeof(int)) != hipSuccess) return fail(HR_EHIP, "hr_set_renderer: memset");
    return HR_OK;
}

int hr_set_tiles(hr_scene* s, int32_t tile_w_log2, int32_t bin_log2)
{
    if (!s) return fail(HR_EINVAL, "hr_set_tiles: null scene");
    return set_tiles(s, tile_w_log2, bin_log2);
}

int hr_get_tiles(const hr_scene* s, int32_t* out_host)
{
    if (!s || !out_host) return fail(HR_EINVAL, "hr_get_tiles: null argument");
    out_host[0] = s->ts.tw_log2;
    out_host[1] = s->ts.th_log2;
    out_host[2] = s->bin_log2;
    return HR_OK;
}

int hr_get_grid(const hr_scene* s, int32_t* blocks_host)
{
    if (!s || !blocks_host) return fail(HR_EINVAL, "hr_get_grid: null argument");
    blocks_host[0] = s->render_blocks;
    blocks_host[1] = s->adjoint_blocks;
    return HR_OK;
}

int hr_tune(hr_scene* s, const hr_state* state, int32_t reps, int32_t* blocks_host, void* stream)
{
    if (!s) return fail(HR_EINVAL, "hr_tune: null scene");
    int rc = check_state(state, "hr_tune");
    if (rc) return rc;
    if (reps < 1 || reps > 100) return fail(HR_EINVAL, "hr_tune: reps must be 1..100");
    hipStream_t st = (hipStream_t)stream;
    const hr_state& q = *state;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(HR_EHIP, "hr_tune: hipEventCreate failed");
    const bool timing = s->timing;
    s->timing = false;
    // the candidates' results are discarded; the iteration index stays on the host
    auto run = [&](bool adjoint) -> int {
        int r = launch(s, "k_skin", k_skin, dim3(s->skin_blocks, s->n_hands), dim3(128), 0, st, s->mesh,
                       (const float*)q.params, q.verts, (float*)nullptr, (int*)nullptr, (float*)nullptr);
        if (!r) r = render_impl(s, q.verts, q.albedo, q.background, 0, nullptr, q.image, nullptr, st);
        if (!r && adjoint) {
            r = loss_impl(s, q.image, q.target, q.mask, q.loss, q.dimage, st);
            if (!r)
                r = backward_impl(s, q.params, q.verts, q.albedo, q.background, q.dimage, 0, nullptr,
                                  HR_GRAD_INTERIOR | HR_REUSE_GEOMETRY, q.grad_params, q.grad_albedo, nullptr,
                                  nullptr, st);
        }
        return r;
    };
    auto measure = [&](bool adjoint, float* ms) -> int {
        int r = run(adjoint);   // warm
        if (!r && hipEventRecord(e0, st) != hipSuccess) r = fail(HR_EHIP, "hr_tune: event");
        for (int i = 0; i < reps && !r; ++i) r = run(adjoint);
        if (!r && hipEventRecord(e1, st) != hipSuccess) r = fail(HR_EHIP, "hr_tune: event");
        if (!r && hipEventSynchronize(e1) != hipSuccess) r = fail(HR_EHIP, "hr_tune: sync");
        if (!r) (void)hipEventElapsedTime(ms, e0, e1);
        return r;
    };
    // first the wave-tile shape and the bin size (render + adjoint at the
    // current grids), then the render grid, then the adjoint grid
    {
        const int ppw = s->ts.tw_log2 + s->ts.th_log2;
        int best_tw = s->ts.tw_log2, best_lb = s->bin_log2;
        float best_ms = 3.4e38f;
        for (int lb = kMinBinLog2; lb <= kMaxBinLog2 && !rc; ++lb)
            for (int tw = std::max(0, ppw - lb); tw <= std::min(ppw, lb) && !rc; ++tw) {
                rc = set_tiles(s, tw, lb);
                float ms = 0.0f;
                if (!rc) rc = measure(true, &ms);
                if (!rc && ms < best_ms) { best_ms = ms; best_tw = tw; best_lb = lb; }
            }
        if (!rc) rc = set_tiles(s, best_tw, best_lb);
    }
    static const int kCand[] = {256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096};
    float best = 0.0f;
    int best_r = s->render_blocks, best_a = s->adjoint_blocks;
    for (int pass = 0; pass < 2 && !rc; ++pass) {
        const bool adjoint = pass == 1;
        best = 3.4e38f;
        int last = -1;
        for (int c : kCand) {
            const int b = std::min(c, s->max_blocks);
            if (b == last) continue;
            last = b;
            if (adjoint) s->adjoint_blocks = b; else s->render_blocks = b;
            float ms = 0.0f;
            rc = measure(adjoint, &ms);
            if (rc) break;
            if (ms < best) { best = ms; if (adjoint) best_a = b; else best_r = b; }
        }
        // the adjoint pass times render + adjoint with the chosen render grid
        s->render_blocks = best_r;
        s->adjoint_blocks = best_a;
    }
    s->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (blocks_host) { blocks_host[0] = s->render_blocks; blocks_host[1] = s->adjoint_blocks; }
    return HR_OK;
}

int hr_proposal_set(hr_scene* s, const hr_proposal_config* cfg, const float* theta_host)
{
    if (!s || !cfg) return fail(HR_EINVAL, "hr_proposal_set: null argument");
    if (cfg->kind != HR_PROPOSAL_LENGTH && cfg->kind != HR_PROPOSAL_LEARNED)
        return fail(HR_EINVAL, "hr_proposal_set: unknown kind");
    if (!(cfg->eps > 0.0f && cfg->eps <= 1.0f)) return fail(HR_EINVAL, "hr_proposal_set: eps must be in (0,1]");
    if (!(cfg->ema >= 0.0f && cfg->ema < 1.0f)) return fail(HR_EINVAL, "hr_proposal_set: ema must be in [0,1)");
    if (!(cfg->lr >= 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
        !(cfg->adam_eps > 0.0f))
        return fail(HR_EINVAL, "hr_proposal_set: bad optimiser settings");
    if (cfg->kind == HR_PROPOSAL_LEARNED && s->E > kPropMaxEdges)
        return fail(HR_EUNSUPPORTED, "hr_proposal_set: more than %d edges", kPropMaxEdges);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(HR_EHIP, "hr_proposal_set: %s", hipGetErrorString(e));
    PropDev& P = s->prop;
    const size_t nve = (size_t)s->n_views * s->E;
    if (!s->prop_alloc) {
        int rc = HR_OK;
        if (!rc) rc = s->upload<float>(&P.theta, nullptr, kMlpParams);
        if (!rc) rc = s->upload<float>(&P.m, nullptr, kMlpParams);
        if (!rc) rc = s->upload<float>(&P.v, nullptr, kMlpParams);
        if (!rc) rc = s->upload<float>(&P.grad, nullptr, kMlpParams);
        if (!rc) rc = s->upload<int>(&P.step, nullptr, 1);
        if (!rc) rc = s->upload<s4v>(&P.w1p, nullptr, 4 * 64);
        if (!rc) rc = s->upload<s4v>(&P.w2p, nullptr, 16 * 64);
        if (!rc) rc = s->upload<s4v>(&P.w2bp, nullptr, 16 * 64);
        if (!rc) rc = s->upload<float>(&P.fb, nullptr, kFbSize);
        if (!rc) rc = s->upload<float>(&P.z, nullptr, nve);
        if (!rc) rc = s->upload<s4v>(&P.feat, nullptr, nve * 4);
        if (!rc) rc = s->upload<float>(&P.stat_a, nullptr, nve);
        if (!rc) rc = s->upload<float>(&P.stat_dc, nullptr, nve * 4);
        if (!rc) rc = s->upload<float>(&P.ema, nullptr, nve * 4);
        if (!rc) rc = s->upload<float>(&s->fit_z, nullptr, kFitMaxRows);
        if (!rc) rc = s->upload<unsigned short>(&P.list, nullptr, nve);
        if (!rc) rc = s->upload<int>(&P.nlist, nullptr, (size_t)s->n_views);
        if (!rc) rc = s->upload<double>(&P.vstat, nullptr, 2 * (size_t)s->n_views);
        if (!rc) rc = s->upload<int>(&P.vcount, nullptr, (size_t)s->n_views);
        if (!rc) rc = s->upload<int>(&P.tcount, nullptr, 1);
        if (rc) return rc;
        s->prop_alloc = true;
        e = hipMemset(P.theta, 0, sizeof(float) * kMlpParams);
        if (e == hipSuccess) e = hipMemset(P.feat, 0, sizeof(s4v) * nve * 4);
        if (e == hipSuccess) e = hipMemset(P.nlist, 0, sizeof(int) * s->n_views);
        if (e == hipSuccess) e = hipMemset(P.vcount, 0, sizeof(int) * s->n_views);
        if (e == hipSuccess) e = hipMemset(P.tcount, 0, sizeof(int));
        if (e != hipSuccess) return fail(HR_EHIP, "hr_proposal_set: %s", hipGetErrorString(e));
    }
    if (theta_host) {
        e = hipMemcpy(P.theta, theta_host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(HR_EHIP, "hr_proposal_set: %s", hipGetErrorString(e));
    }
    // fresh optimiser state, statistics and colour-jump averages
    e = hipMemset(P.m, 0, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMemset(P.v, 0, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMemset(P.grad, 0, sizeof(float) * kMlpParams);
    if (e == hipSuccess) e = hipMemset(P.step, 0, sizeof(int));
    if (e == hipSuccess) e = hipMemset(P.z, 0, sizeof(float) * nve);
    if (e == hipSuccess) e = hipMemset(P.stat_a, 0, sizeof(float) * nve);
    if (e == hipSuccess) e = hipMemset(P.stat_dc, 0, sizeof(float) * nve * 4);
    if (e == hipSuccess) e = hipMemset(P.ema, 0, sizeof(float) * nve * 4);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_proposal_set: %s", hipGetErrorString(e));
    P.eps = cfg->eps; P.ema_beta = cfg->ema; P.lr = cfg->lr;
    P.beta1 = cfg->beta1; P.beta2 = cfg->beta2; P.adam_eps = cfg->adam_eps;
    P.split = std::max(1, std::min(8, 256 / s->n_views));
    s->prop_kind = cfg->kind;
    hipLaunchKernelGGL(k_proposal_pack, dim3(1), dim3(256), 0, (hipStream_t)0, P);
    int rc = check_launch("hr_proposal_set");
    if (rc) return rc;
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(HR_EHIP, "hr_proposal_set: %s", hipGetErrorString(e));
    return HR_OK;
}

static int need_prop(const hr_scene* s, const char* who)
{
    if (!s) return fail(HR_EINVAL, "%s: null scene", who);
    if (!s->prop_alloc) return fail(HR_EINVAL, "%s: no proposal set on this scene (hr_proposal_set)", who);
    return HR_OK;
}

int hr_proposal_get(hr_scene* s, float* theta_host, void* stream)
{
    int rc = need_prop(s, "hr_proposal_get");
    if (rc) return rc;
    if (!theta_host) return fail(HR_EINVAL, "hr_proposal_get: null argument");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipMemcpy(theta_host, s->prop.theta, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_proposal_get: %s", hipGetErrorString(e));
    return HR_OK;
}

int hr_proposal_override(hr_scene* s, const float* z)
{
    int rc = need_prop(s, "hr_proposal_override");
    if (rc) return rc;
    s->prop.z_override = z;
    return HR_OK;
}

int hr_proposal_train(hr_scene* s, void* stream)
{
    int rc = need_prop(s, "hr_proposal_train");
    if (rc) return rc;
    return proposal_train_impl(s, (hipStream_t)stream);
}

int hr_proposal_features(hr_scene* s, float* feats, void* stream)
{
    int rc = need_prop(s, "hr_proposal_features");
    if (rc) return rc;
    if (!feats) return fail(HR_EINVAL, "hr_proposal_features: null argument");
    const long long rows = (long long)s->n_views * s->E;
    return launch(s, "k_proposal_read_feat", k_proposal_read_feat,
                  dim3((unsigned)std::min<long long>(4096, (rows * 16 + 255) / 256)), dim3(256), 0,
                  (hipStream_t)stream, (const s4v*)s->prop.feat, (const EdgeRec*)s->edge_rec, rows, feats);
}

int hr_proposal_stats(hr_scene* s, float* z, uint32_t* wq, float* a, float* dc, void* stream)
{
    int rc = need_prop(s, "hr_proposal_stats");
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t rows = (size_t)s->n_views * s->E;
    hipError_t e = hipSuccess;
    if (z) e = hipMemcpyAsync(z, s->prop.z, sizeof(float) * rows, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && a) e = hipMemcpyAsync(a, s->prop.stat_a, sizeof(float) * rows, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && dc)
        e = hipMemcpyAsync(dc, s->prop.stat_dc, sizeof(float) * rows * 4, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_proposal_stats: %s", hipGetErrorString(e));
    if (wq)
        return launch(s, "k_proposal_read_wq", k_proposal_read_wq,
                      dim3((unsigned)std::min<size_t>(4096, (rows + 255) / 256)), dim3(256), 0, st,
                      (const EdgeRec*)s->edge_rec, (long long)rows, wq);
    return HR_OK;
}

int hr_proposal_eval(hr_scene* s, const float* X, int32_t n, float* z, void* stream)
{
    int rc = need_prop(s, "hr_proposal_eval");
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!X || !z))) return fail(HR_EINVAL, "hr_proposal_eval: bad argument");
    if (n == 0) return HR_OK;
    return launch(s, "k_proposal_eval", k_proposal_eval, dim3((unsigned)((n + 63) / 64)), dim3(256), 0,
                  (hipStream_t)stream, s->prop, X, (int)n, z);
}

int hr_proposal_fit(hr_scene* s, const float* X, const uint32_t* w, const float* a, int32_t n, float* grad,
                    int32_t apply, void* stream)
{
    int rc = need_prop(s, "hr_proposal_fit");
    if (rc) return rc;
    if (n < 1 || n > kFitMaxRows || !X || !w || !a)
        return fail(HR_EINVAL, "hr_proposal_fit: need 1..%d rows and non-null X, w, a", kFitMaxRows);
    hipStream_t st = (hipStream_t)stream;
    rc = launch(s, "k_proposal_eval", k_proposal_eval, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, st, s->prop, X,
                (int)n, s->fit_z);
    if (!rc)
        rc = launch(s, "k_proposal_fit", k_proposal_fit, dim3(1), dim3(256), 0, st, s->prop, X, w, a,
                    (const float*)s->fit_z, (int)n, grad, (int)(apply != 0));
    if (!rc && apply) rc = launch(s, "k_proposal_adam", k_proposal_adam, dim3(1), dim3(256), 0, st, s->prop);
    return rc;
}

// ---------------------------------------------------------------------------
// full data term
// ---------------------------------------------------------------------------

int hr_data_term_set(hr_scene* s, const hr_data_term* cfg)
{
    if (!s || !cfg) return fail(HR_EINVAL, "hr_data_term_set: null argument");
    if (!(cfg->w_edge >= 0.0f) || !std::isfinite(cfg->w_edge) || !(cfg->low >= 0.0f) || !(cfg->high >= cfg->low) ||
        !std::isfinite(cfg->high))
        return fail(HR_EINVAL, "hr_data_term_set: need w_edge >= 0 and 0 <= low <= high (finite)");
    DataTermDev& d = s->dt;
    if (!s->dt_alloc) {
        const hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return fail(HR_EHIP, "hr_data_term_set: %s", hipGetErrorString(e));
        const size_t P = (size_t)s->n_pixels;
        int rc = HR_OK;
        if (!rc) rc = s->upload<double>(&d.w5, nullptr, 25);
        if (!rc) rc = s->upload<double>(&d.w11, nullptr, 121);
        if (!rc) rc = s->upload<double>(&d.w11s, nullptr, 11);
        if (!rc) rc = s->upload<double>(&d.w5s, nullptr, 5);
        double* bufs[10];
        for (int k = 0; k < 10 && !rc; ++k) rc = s->upload<double>(&bufs[k], nullptr, P);
        if (!rc) rc = s->upload<uint8_t>(&d.flags, nullptr, P);
        if (!rc) rc = s->upload<double>(&d.vsum, nullptr, 2 * (size_t)s->n_views);
        if (!rc) rc = s->upload<double>(&d.gT, nullptr, 9 * (size_t)s->n_views);
        if (rc) return rc;
        d.grey = bufs[0]; d.sm = bufs[1]; d.gx = bufs[2]; d.gy = bufs[3]; d.mag = bufs[4];
        d.edge = bufs[5]; d.blur = bufs[6]; d.g1 = bufs[7]; d.g2 = bufs[8]; d.gb = bufs[9];
        // normalised Gaussian weights exp(-(i^2 + j^2) / (2 sigma^2))
        auto gauss = [](int size, double sigma, double* host) {
            const double c = (size - 1) / 2.0;
            double sum = 0.0;
            for (int i = 0; i < size; ++i)
                for (int j = 0; j < size; ++j) {
                    const double di = i - c, dj = j - c;
                    host[size * i + j] = std::exp(-(di * di + dj * dj) / (2.0 * sigma * sigma));
                    sum += host[size * i + j];
                }
            for (int k = 0; k < size * size; ++k) host[k] /= sum;
        };
        double w5[25], w11[121], w11s[11], sum1 = 0.0;
        gauss(5, 1.0, w5);
        gauss(11, 5.0, w11);
        // the blur's factor: w11[i][j] = w11s[i] w11s[j]
        for (int k = 0; k < 11; ++k) {
            w11s[k] = std::exp(-(double)((k - 5) * (k - 5)) / 50.0);
            sum1 += w11s[k];
        }
        for (int k = 0; k < 11; ++k) w11s[k] /= sum1;
        // the smoothing's factor: w5[i][j] = w5s[i] w5s[j]
        double w5s[5], sum5 = 0.0;
        for (int k = 0; k < 5; ++k) {
            w5s[k] = std::exp(-(double)((k - 2) * (k - 2)) / 2.0);
            sum5 += w5s[k];
        }
        for (int k = 0; k < 5; ++k) w5s[k] /= sum5;
        hipError_t e2 = hipMemcpy(d.w5, w5, sizeof(w5), hipMemcpyHostToDevice);
        if (e2 == hipSuccess) e2 = hipMemcpy(d.w11, w11, sizeof(w11), hipMemcpyHostToDevice);
        if (e2 == hipSuccess) e2 = hipMemcpy(d.w11s, w11s, sizeof(w11s), hipMemcpyHostToDevice);
        if (e2 == hipSuccess) e2 = hipMemcpy(d.w5s, w5s, sizeof(w5s), hipMemcpyHostToDevice);
        if (e2 != hipSuccess) return fail(HR_EHIP, "hr_data_term_set: %s", hipGetErrorString(e2));
        s->dt_alloc = true;
    }
    d.w_e = cfg->w_edge;
    d.low = cfg->low;
    d.high = cfg->high;
    return HR_OK;
}

static DtArgs dt_args(hr_scene* s, const float* image, const float* T)
{
    DtArgs a;
    a.chunks = s->chunks; a.views = s->views; a.image = image; a.T = T;
    a.target = nullptr; a.target_edges = nullptr; a.mask = nullptr; a.view_scale = s->view_scale;
    a.d = s->dt;
    return a;
}

// stages of B(Canny(T R)) up to the blur
static int dt_canny(hr_scene* s, const DtArgs& a, hipStream_t st)
{
    const dim3 g(s->n_chunks, kDtSplit), b(256);
    int rc = launch(s, "k_dt_grey", k_dt_grey, g, b, 0, st, a);
    if (!rc) rc = launch(s, "k_dt_smooth", k_dt_smooth, g, b, 0, st, a);
    if (!rc) rc = launch(s, "k_dt_grad", k_dt_grad, g, b, 0, st, a);
    if (!rc) rc = launch(s, "k_dt_suppress", k_dt_suppress, g, b, 0, st, a);
    if (!rc) rc = launch(s, "k_dt_hyst", k_dt_hyst, g, b, 0, st, a);
    return rc;
}

int hr_edge_map(hr_scene* s, const float* image, const float* T, float* edge_map, void* stream)
{
    if (!s || !image || !edge_map) return fail(HR_EINVAL, "hr_edge_map: null argument");
    if (!s->dt_alloc) return fail(HR_EINVAL, "hr_edge_map: call hr_data_term_set first");
    const hipStream_t st = (hipStream_t)stream;
    const DtArgs a = dt_args(s, image, T);
    int rc = dt_canny(s, a, st);
    if (!rc) rc = launch(s, "k_dt_blur_col", k_dt_blur_col, dim3(s->n_chunks, kDtSplit), dim3(256), 0, st, a, s->dt.g1);
    if (!rc)
        rc = launch(s, "k_dt_blur", k_dt_blur<false>, dim3(s->n_chunks, kDtSplit), dim3(256), 0, st, a, (const double*)s->dt.g1,
                    edge_map);
    return rc;
}

int hr_loss_full(hr_scene* s, const float* image, const float* T, const float* target, const float* target_edges,
                 const uint8_t* mask, float* loss, float* dimage, float* grad_T, float* edge_map, void* stream)
{
    if (!s || !image || !target || !target_edges || !loss || !dimage)
        return fail(HR_EINVAL, "hr_loss_full: null argument");
    if (!s->dt_alloc) return fail(HR_EINVAL, "hr_loss_full: call hr_data_term_set first");
    const hipStream_t st = (hipStream_t)stream;
    DtArgs a = dt_args(s, image, T);
    a.target = target; a.target_edges = target_edges; a.mask = mask;
    int rc = launch(s, "k_dt_zero", k_dt_zero, dim3(1), dim3(256), 0, st, s->dt.vsum, 2 * s->n_views);
    if (!rc) rc = launch(s, "k_dt_zero", k_dt_zero, dim3(1), dim3(256), 0, st, s->dt.gT, 9 * s->n_views);
    if (!rc) rc = launch(s, "k_dt_scale", k_dt_scale, dim3(s->n_views), dim3(256), 0, st, (const ViewDev*)s->views, mask,
                         s->view_scale);
    if (!rc) rc = dt_canny(s, a, st);
    const dim3 g(s->n_chunks, kDtSplit), b(256);
    // the column pass writes g1 (free until the backward); the backward's
    // row pass writes the edge map's buffer (no longer read)
    if (!rc) rc = launch(s, "k_dt_blur_col", k_dt_blur_col, g, b, 0, st, a, s->dt.g1);
    if (!rc) rc = launch(s, "k_dt_blur", k_dt_blur<true>, g, b, 0, st, a, (const double*)s->dt.g1, edge_map);
    if (!rc) rc = launch(s, "k_dt_bwd_blur_row", k_dt_bwd_blur_row, g, b, 0, st, a, s->dt.edge);
    if (!rc) rc = launch(s, "k_dt_bwd_edge", k_dt_bwd_edge, g, b, 0, st, a, (const double*)s->dt.edge);
    if (!rc) rc = launch(s, "k_dt_bwd_sobel", k_dt_bwd_sobel, g, b, 0, st, a, s->dt.sm);
    // the smoothing's transpose: row pass into the Canny map's buffer (free by now), column pass in the final kernel
    if (!rc) rc = launch(s, "k_dt_bwd_smooth_row", k_dt_bwd_smooth_row, g, b, 0, st, a, (const double*)s->dt.sm, s->dt.edge);
    if (!rc) rc = launch(s, "k_dt_bwd_final", k_dt_bwd_final, g, b, 0, st, a, (const double*)s->dt.edge, dimage);
    if (!rc)
        rc = launch(s, "k_dt_finish", k_dt_finish, dim3(1), dim3(256), 0, st, a, (const int*)s->hand_view_off,
                    (const int*)s->hand_views, s->n_hands, s->n_views, loss, grad_T);
    return rc;
}

int hr_compose_albedo(hr_scene* s, const float* low, int32_t L, const float* high, float* albedo, void* stream)
{
    if (!s || !low || !high || !albedo) return fail(HR_EINVAL, "hr_compose_albedo: null argument");
    const int th = s->cfg.tex_h, tw = s->cfg.tex_w;
    if (L < 1 || th % L || tw % L) return fail(HR_ESHAPE, "hr_compose_albedo: %d does not divide %d x %d", L, th, tw);
    const long long n = (long long)s->n_hands * th * tw * 3;
    const unsigned blocks = (unsigned)std::min<long long>(4096, (n + 255) / 256);
    return launch(s, "k_compose_albedo", k_compose_albedo, dim3(blocks), dim3(256), 0, (hipStream_t)stream, low, L, high,
                  albedo, th, tw, n);
}

int hr_albedo_low_grad(hr_scene* s, const float* grad_albedo, int32_t L, float* grad_low, void* stream)
{
    if (!s || !grad_albedo || !grad_low) return fail(HR_EINVAL, "hr_albedo_low_grad: null argument");
    const int th = s->cfg.tex_h, tw = s->cfg.tex_w;
    if (L < 1 || th % L || tw % L) return fail(HR_ESHAPE, "hr_albedo_low_grad: %d does not divide %d x %d", L, th, tw);
    return launch(s, "k_albedo_low_grad", k_albedo_low_grad, dim3(s->n_hands * L * L), dim3(256), 0, (hipStream_t)stream,
                  grad_albedo, L, th, tw, grad_low);
}

int hr_adam(hr_scene* s, float* x, const float* g, float* m, float* v, int64_t n, int32_t t, float lr, float lo,
            float hi, const hr_adam_config* cfg, void* stream)
{
    if (!s || !x || !g || !m || !v || !cfg) return fail(HR_EINVAL, "hr_adam: null argument");
    if (n < 0 || t < 1 || !(lo <= hi)) return fail(HR_EINVAL, "hr_adam: need n >= 0, t >= 1, lo <= hi");
    if (n == 0) return HR_OK;
    const float bc1 = (float)(1.0 - std::pow((double)cfg->beta1, (double)t));
    const float bc2 = (float)(1.0 - std::pow((double)cfg->beta2, (double)t));
    const unsigned blocks = (unsigned)std::min<long long>(4096, (n + 255) / 256);
    return launch(s, "k_adam_plain", k_adam_plain, dim3(blocks), dim3(256), 0, (hipStream_t)stream, x, g, m, v,
                  (long long)n, lr, cfg->beta1, cfg->beta2, cfg->eps, bc1, bc2, lo, hi);
}

int hr_edge_stats(hr_scene* s, uint64_t* total_host, int64_t* budget_host, void* stream)
{
    if (!s || !total_host || !budget_host) return fail(HR_EINVAL, "hr_edge_stats: null argument");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess)
        e = hipMemcpy(total_host, s->edge_total, sizeof(uint64_t) * s->n_views, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(budget_host, s->edge_budget, sizeof(int64_t) * s->n_views, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(HR_EHIP, "hr_edge_stats: %s", hipGetErrorString(e));
    return HR_OK;
}

}  // extern "C"
