// Device-side building blocks of the handrt kernels (gfx950, wave64).
//
// Float32 decisions (closest hit, silhouette classification, edge sample
// placement) are written with an explicit evaluation order and the library is
// compiled with -ffp-contract=off, so each decision rounds exactly as written:
// a float64 host evaluation that follows the same published algorithms in
// float32 reaches the same integer results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hr {

constexpr int kMaxStack = 24;       // traversal stack entries per lane
constexpr int kLeafMax = 4;         // triangles per leaf
constexpr int kThreads = 256;       // threads per block of the ray-tracing kernels
constexpr int kEdgeBlocks = 256;    // blocks of edge samples in the backward launch
constexpr int kMaxTraceBlocks = 16384;  // largest ray-tracing grid
constexpr int kWin = 16;            // texel window (per row of 16 lanes) of the colour-map gradient: kWin^2 weights
constexpr int kWinRGB = 9;          // ... or kWinRGB^2 RGB texels (3 kWinRGB^2 <= kWin^2)
constexpr int kWaveWin = 4 * kWin * kWin;   // floats of one wave's four row windows

// ---------------------------------------------------------------------------
// records in device memory
// ---------------------------------------------------------------------------

// read-only global data addressed as constant memory: wave-uniform loads of
// it become scalar loads
typedef const __attribute__((address_space(4))) float ConstF;
typedef const __attribute__((address_space(4))) int ConstI;

struct ViewDev {            // one camera (see hr_camera)
    float R[9];
    float o[3];
    float fx, fy, cx, cy;
    int W, H, hand;
    uint32_t sid;           // sample-stream id (Philox counter word of the view)
    int bin0, nbx;          // first screen bin of the view in the scene's bin arrays, bins per row
    long long pix0;         // first pixel in packed buffers
};

constexpr int kBinLog2 = 4;         // default screen bins of 16 x 16 pixels (wave tiles never straddle one)
constexpr int kMinBinLog2 = 3, kMaxBinLog2 = 5;   // bin sizes the tuner may choose (8 .. 32 pixels)
constexpr int kMaxBinsLds = 8192;   // bins of a view counted in LDS (larger views traverse the hierarchy)
constexpr int kMaxBands = 16;       // depth bands per bin (fewer for views with many bins)
constexpr int kMaxBinCells = 8192;  // (bin, band) cells counted in LDS
// A view's record through the scalar cache (views are never written by a
// launch; the index must be wave-uniform).
__device__ __forceinline__ ViewDev load_view(const ViewDev* views, int i)
{
    ViewDev v;
    const ConstI* src = (const ConstI*)(views + i);
    int* dst = reinterpret_cast<int*>(&v);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(ViewDev) / 4); ++k) dst[k] = src[k];
    return v;
}

struct alignas(16) Node {   // internal node: bounds of both children
    float lo0[3], hi0[3], lo1[3], hi1[3];
    int child[2];           // >= 0 internal node, < 0 leaf: ~(start << 3 | count)
    int pad[2];
};


struct alignas(16) Tri {    // triangle in leaf order
    float v[9];
    int face, i0, i1, i2;
    int pad[3];
};

struct alignas(16) EdgeRec {  // silhouette edge of one view (float32)
    float ax, ay, bx, by;     // projected endpoints
    float t0, t1;             // clipped parameter interval
    uint32_t w;               // quantised length, 1/256 px (0 = not sampled)
    uint32_t wq;              // sampling weight (= w for length-proportional sampling)
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------

struct U64x4 { uint64_t x[4]; };

__device__ __forceinline__ U64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t y0 = hi1 ^ c1 ^ k0;
        uint64_t y2 = hi0 ^ c3 ^ k1;
        c0 = y0; c1 = lo1; c2 = y2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    U64x4 o;
    o.x[0] = c0; o.x[1] = c1; o.x[2] = c2; o.x[3] = c3;
    return o;
}

__device__ __forceinline__ float u24_lo(uint64_t r) { return (float)((uint32_t)r >> 8) * 0x1p-24f; }
__device__ __forceinline__ float u24_hi(uint64_t r) { return (float)(r >> 40) * 0x1p-24f; }

// A stored camera sample: its random word (bits 8..31 and 40..63 are u and
// v) with the hit's leaf slot (int16, -1 miss) in the bits u and v leave out
// (0..7 low byte, 32..39 high byte).
__device__ __forceinline__ uint64_t hit_record(uint64_t wd, int slot)
{
    const uint64_t s16 = (uint64_t)(uint16_t)slot;
    return (wd & 0xFFFFFF00FFFFFF00ull) | (s16 & 0xFFu) | ((s16 >> 8) << 32);
}

__device__ __forceinline__ int hit_record_slot(uint64_t rec)
{
    return (int)(int16_t)(uint16_t)((rec & 0xFFu) | ((rec >> 24) & 0xFF00u));
}

constexpr uint64_t kDomainCamera = 0;
constexpr uint64_t kDomainEdge = 1;

// ---------------------------------------------------------------------------
// rays and the watertight test (Woop, Benthin, Wald, JCGT 2013)
// ---------------------------------------------------------------------------

struct Ray {
    float o[3], d[3];
    int kx, ky, kz;
    float Sx, Sy, Sz;
    float inv[3];           // 1/d for the slab test (|d| clamped away from 0)
    float oi[3];            // o * inv: a slab plane's t is one fused multiply-add
};

// component k of a: two selects, never a branch (lanes of a wave may differ
// in k, and a branch per component costs a run of exec-mask instructions)
__device__ __forceinline__ float comp(const float* a, int k)
{
    const float a0 = a[0], a1 = a[1], a2 = a[2];
    const float r = k == 1 ? a1 : a0;
    return k == 2 ? a2 : r;
}

__device__ __forceinline__ void ray_setup(Ray& r)
{
    int kz = 0;
    if (fabsf(r.d[1]) > fabsf(r.d[kz])) kz = 1;
    if (fabsf(r.d[2]) > fabsf(comp(r.d, kz))) kz = 2;
    int kx = kz + 1; if (kx == 3) kx = 0;
    int ky = kx + 1; if (ky == 3) ky = 0;
    float dz = comp(r.d, kz);
    if (dz < 0.0f) { int t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.Sx = comp(r.d, kx) / dz;
    r.Sy = comp(r.d, ky) / dz;
    r.Sz = 1.0f / dz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float dk = r.d[k];
        if (fabsf(dk) < 1e-20f) dk = dk < 0.0f ? -1e-20f : 1e-20f;
        // the hardware reciprocal (within 1 ulp): the slab test only culls,
        // and a relative error of 1e-7 in t stays far inside the bounds'
        // padding; the watertight test's Sx, Sy, Sz keep exact divisions
        r.inv[k] = __builtin_amdgcn_rcpf(dk);
        r.oi[k] = r.o[k] * r.inv[k];
    }
}

// ray through screen point (sx, sy): origin at the camera centre, direction R^T dc
__device__ __forceinline__ void ray_screen(const ViewDev& c, float sx, float sy, Ray& r)
{
    float dcx = (sx - c.cx) / c.fx;
    float dcy = (sy - c.cy) / c.fy;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float a = c.R[k] * dcx;
        float b = c.R[3 + k] * dcy;
        r.d[k] = (a + b) + c.R[6 + k];
        r.o[k] = c.o[k];
    }
    ray_setup(r);
}

// returns true and (t, U, V, W, det) when the ray hits the triangle with t > 0
__device__ __forceinline__ bool watertight(const Ray& r, const float* v0, const float* v1,
                                           const float* v2, float& t_out, float& U_out,
                                           float& V_out, float& W_out, float& det_out)
{
    float A[3], B[3], C[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        A[k] = v0[k] - r.o[k];
        B[k] = v1[k] - r.o[k];
        C[k] = v2[k] - r.o[k];
    }
    const float Akx = comp(A, r.kx), Aky = comp(A, r.ky), Akz = comp(A, r.kz);
    const float Bkx = comp(B, r.kx), Bky = comp(B, r.ky), Bkz = comp(B, r.kz);
    const float Ckx = comp(C, r.kx), Cky = comp(C, r.ky), Ckz = comp(C, r.kz);
    float Ax = Akx - r.Sx * Akz;
    float Ay = Aky - r.Sy * Akz;
    float Bx = Bkx - r.Sx * Bkz;
    float By = Bky - r.Sy * Bkz;
    float Cx = Ckx - r.Sx * Ckz;
    float Cy = Cky - r.Sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        double CxBy = (double)Cx * (double)By, CyBx = (double)Cy * (double)Bx;
        double AxCy = (double)Ax * (double)Cy, AyCx = (double)Ay * (double)Cx;
        double BxAy = (double)Bx * (double)Ay, ByAx = (double)By * (double)Ax;
        U = (float)(CxBy - CyBx);
        V = (float)(AxCy - AyCx);
        W = (float)(BxAy - ByAx);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = (U + V) + W;
    if (det == 0.0f) return false;
    float Az = r.Sz * Akz;
    float Bz = r.Sz * Bkz;
    float Cz = r.Sz * Ckz;
    float T = (U * Az + V * Bz) + W * Cz;
    float t = T / det;
    if (!(t > 0.0f)) return false;
    t_out = t; U_out = U; V_out = V; W_out = W; det_out = det;
    return true;
}

struct Hit {
    int face;         // -1: miss
    int slot;         // leaf-order index of the triangle
    float t;
};

// Surface point of a hit, with barycentrics recomputed in float64 from the
// exact sample ray: the float32 test decides the triangle, float64 gives the
// position on it (well conditioned even at grazing incidence).
struct Surf {
    int face;         // face id of the triangle
    int i0, i1, i2;
    float b0, b1, b2;
    double tu, tv;    // texture coordinates (float64: texel positions stay exact)
    float v[9];       // triangle vertices
    double d[3];      // float64 ray direction (unnormalised, camera depth scale)
    double pv[3];     // d x (v2 - v0) and 1 / det of the solve (reused by the adjoint)
    double idet;
};

__device__ __forceinline__ bool slab(const Ray& r, const float* lo, const float* hi, float tmax_in,
                                     float& tmin_out)
{
    // t of the plane x = lo as lo / d - o / d: the error of the rounded o / d
    // (half an ulp of it) stays far below the bounds' padding (1e-5 + 1e-6 |x|
    // in x, i.e. (1e-5 + 1e-6 |x|) / |d| in t) for origins within metres
    float tx0 = __builtin_fmaf(lo[0], r.inv[0], -r.oi[0]), tx1 = __builtin_fmaf(hi[0], r.inv[0], -r.oi[0]);
    float ty0 = __builtin_fmaf(lo[1], r.inv[1], -r.oi[1]), ty1 = __builtin_fmaf(hi[1], r.inv[1], -r.oi[1]);
    float tz0 = __builtin_fmaf(lo[2], r.inv[2], -r.oi[2]), tz1 = __builtin_fmaf(hi[2], r.inv[2], -r.oi[2]);
    float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tmax_in));
    tmin_out = tmin;
    return tmin <= tmax;
}

// Work counters of one traversal (only maintained when COUNT is true).
struct TraceCount {
    unsigned nodes = 0, tris = 0;       // the ray's own work: nodes whose box it enters, triangles of
                                        // leaves whose box it enters
    unsigned nodes_w = 0, tris_w = 0;   // packet traversal: node visits and triangle tests executed
                                        // while this lane was active (the union of the wave's rays)
};

// Closest hits of the rays of one wave by a single traversal order: the wave
// visits a node when any active lane's ray enters the node's box before that
// lane's best hit so far (the union of the per-ray traversals), and every lane
// keeps its own closest (t, face id).  A lane therefore tests every triangle
// its own traversal would test (plus possibly others, which cannot beat its
// closest hit), so each result equals the per-ray traversal's and a brute-force
// loop's.  Meant for coherent rays (all samples of a few adjacent pixels):
// the node and triangle addresses are wave-uniform and the stack is one per
// wave.  Every lane of the wave must call it; inactive lanes take no part.
// `wstack`: this wave's LDS stack (kMaxStack ints).  SFETCH: nodes and
// triangles are fetched through the scalar data cache (reads only; the
// hierarchy is not written during the launch), which suits packets whose
// node sequence is short and shared by many waves (camera rays); incoherent
// packets (silhouette side points) keep vector fetches.
// lane mask of a predicate over the wave (inactive lanes 0)
__device__ __forceinline__ uint64_t wave_mask(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// a wave-uniform pointer held in scalar registers
template <typename T>
__device__ __forceinline__ const T* uniform_ptr(const T* p)
{
    const uint64_t u = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

template <bool COUNT = false, bool SFETCH = false>
__device__ __forceinline__ void trace_wave(const Node* __restrict__ nodes, const Tri* __restrict__ tris,
                                           const Ray& r, bool active, int* wstack, Hit& h,
                                           TraceCount* cnt = nullptr)
{
    h.face = -1;
    h.slot = 0;
    h.t = 0.0f;
    float tb = active ? __builtin_inff() : -__builtin_inff();   // inactive: every box test fails
    int fb = 0x7fffffff;
    int sp = 0;
    int node = 0;
    nodes = uniform_ptr(nodes);
    tris = uniform_ptr(tris);
    // counting: the lanes whose ray entered the current node's box (from the
    // parent's test; the root: every active lane), with a mask per stack entry
    __shared__ uint64_t mstack[COUNT ? kThreads / 64 : 1][COUNT ? kMaxStack : 1];
    const int lane_id = (int)(threadIdx.x & 63);
    uint64_t need = COUNT ? wave_mask(active) : 0ull;
    while (true) {
        if (COUNT) {
            if (active) cnt->nodes_w++;
            if ((need >> lane_id) & 1ull) cnt->nodes++;
        }
        float4 q0, q1, q2;
        int4 q3;
        if (SFETCH) {
            const ConstF* np = (const ConstF*)(nodes + node);
            q0 = make_float4(np[0], np[1], np[2], np[3]);
            q1 = make_float4(np[4], np[5], np[6], np[7]);
            q2 = make_float4(np[8], np[9], np[10], np[11]);
            q3 = make_int4(__float_as_int(np[12]), __float_as_int(np[13]), 0, 0);
        } else {
            const Node& n = nodes[node];
            q0 = *reinterpret_cast<const float4*>(&n.lo0[0]);
            q1 = *reinterpret_cast<const float4*>(&n.hi0[1]);
            q2 = *reinterpret_cast<const float4*>(&n.lo1[2]);
            q3 = *reinterpret_cast<const int4*>(&n.child[0]);
        }
        float lo0[3] = {q0.x, q0.y, q0.z}, hi0[3] = {q0.w, q1.x, q1.y};
        float lo1[3] = {q1.z, q1.w, q2.x}, hi1[3] = {q2.y, q2.z, q2.w};
        const int c0 = __builtin_amdgcn_readfirstlane(q3.x), c1 = __builtin_amdgcn_readfirstlane(q3.y);
        float t0, t1;
        const bool h0 = slab(r, lo0, hi0, tb, t0);
        const bool h1 = slab(r, lo1, hi1, tb, t1);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int code = c == 0 ? c0 : c1;
            const bool hit = c == 0 ? h0 : h1;
            if (code < 0 && wave_mask(hit) != 0) {
                const int lc = ~code;
                const int start = lc >> 3, ncnt = lc & 7;
                if (COUNT && hit) cnt->tris += ncnt;
                if (COUNT && active) cnt->tris_w += ncnt;
                for (int k = 0; k < ncnt; ++k) {
                    float4 p0, p1, p2;
                    if (SFETCH) {
                        const ConstF* tp = (const ConstF*)(tris + start + k);
                        p0 = make_float4(tp[0], tp[1], tp[2], tp[3]);
                        p1 = make_float4(tp[4], tp[5], tp[6], tp[7]);
                        p2 = make_float4(tp[8], tp[9], tp[10], tp[11]);
                    } else {
                        const Tri& tr = tris[start + k];
                        p0 = *reinterpret_cast<const float4*>(&tr.v[0]);
                        p1 = *reinterpret_cast<const float4*>(&tr.v[4]);
                        p2 = *reinterpret_cast<const float4*>(&tr.v[8]);
                    }
                    if (!hit) continue;
                    float v0[3] = {p0.x, p0.y, p0.z};
                    float v1[3] = {p0.w, p1.x, p1.y};
                    float v2[3] = {p1.z, p1.w, p2.x};
                    const int face = __float_as_int(p2.y);
                    float t, U, V, W, det;
                    if (watertight(r, v0, v1, v2, t, U, V, W, det)) {
                        if (t < tb || (t == tb && face < fb)) {
                            tb = t; fb = face;
                            h.face = face;
                            h.slot = start + k;
                            h.t = t;
                        }
                    }
                }
            }
        }
        const uint64_t m0 = c0 >= 0 ? wave_mask(h0 && t0 <= tb) : 0ull;
        const uint64_t m1 = c1 >= 0 ? wave_mask(h1 && t1 <= tb) : 0ull;
        const bool go0 = m0 != 0, go1 = m1 != 0;
        if (go0 && go1) {
            // nearer child first, by majority of the lanes that enter both
            // (the rest of those lanes have t1 < t0: slab entries are not NaN)
            const uint64_t both = m0 & m1;
            const int n01 = __popcll(both & wave_mask(t0 <= t1));
            const int n10 = __popcll(both) - n01;
            const int nearc = n01 >= n10 ? c0 : c1;
            const int farc = n01 >= n10 ? c1 : c0;
            if (COUNT && sp < kMaxStack) mstack[threadIdx.x >> 6][sp] = n01 >= n10 ? m1 : m0;
            if (COUNT) need = n01 >= n10 ? m0 : m1;
            if (sp < kMaxStack) { wstack[sp] = farc; ++sp; }
            node = nearc;
        } else if (go0) {
            node = c0;
            if (COUNT) need = m0;
        } else if (go1) {
            node = c1;
            if (COUNT) need = m1;
        } else {
            if (sp == 0) break;
            --sp;
            node = __builtin_amdgcn_readfirstlane(wstack[sp]);
            if (COUNT) need = mstack[threadIdx.x >> 6][sp];
        }
    }
}

// Closest hits of the camera rays of one wave tile from its screen bin: `ent`
// lists `cnt` leaf slots, `box` holds each slot's padded screen bounds, and
// the tile's rays pass through screen points in [x0, x1] x [y0, y1].  Every
// triangle that a ray of the tile can hit is listed and touches that
// rectangle, and the closest hit is the minimum of (t, face id) over them:
// the result equals a brute-force loop over all triangles.  With NP > 1 the
// calling wave takes only the touching triangles whose rank in the list is
// part mod NP (the minimum over the NP parts is the whole list's).  Before its
// watertight test a triangle is skipped by the wave when no lane can find
// it nearer than its best hit so far: the test computes t as a weighted mean
// of the three vertices' (v[kz] - o[kz]) Sz with non-negative weights, so t
// is at least their minimum, which is computed here with the same rounding
// (times 1 - 1e-6 for the rounding of the mean); a skip therefore never
// drops a hit at or before the lane's best, ties included.  The lanes that
// call it share the list (each loads every n-th entry, n = the calling
// lanes); `active` selects the lanes whose rays are traced.
template <bool COUNT = false, int NP = 1>
__device__ __forceinline__ void trace_bins(const Tri* __restrict__ tris, const uint16_t* __restrict__ ent, int cnt,
                                           const float4* __restrict__ box, float x0, float y0, float x1, float y1,
                                           const Ray& r, bool active, Hit& h, TraceCount* tc = nullptr,
                                           int part = 0)
{
    h.face = -1;
    h.slot = 0;
    h.t = 0.0f;
    float tb = active ? __builtin_inff() : -__builtin_inff();
    int fb = 0x7fffffff;
    tris = uniform_ptr(tris);
    // the calling lanes load the list together: lane of rank k takes entries
    // c0 + k, c0 advancing by their number
    const uint64_t exec = wave_mask(true);
    const int ncall = __popcll(exec);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(exec >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)exec, 0u));
    const float okz = comp(r.o, r.kz);
    int rank_t = 0;   // touching triangles seen (NP > 1)
    // lane-parallel loads of a chunk of entries: each lane fetches its
    // entry's bounds and triangle at once (no dependent fetch per triangle),
    // the loop then broadcasts the touching ones lane by lane
    for (int c0 = 0; c0 < cnt; c0 += ncall) {
        int slot = 0;
        bool touch = false;
        float4 q0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), q1 = q0, q2 = q0;
        if (c0 + rank < cnt) {
            slot = ent[c0 + rank];
            const Tri& tr = tris[slot];
            q0 = *reinterpret_cast<const float4*>(&tr.v[0]);
            q1 = *reinterpret_cast<const float4*>(&tr.v[4]);
            q2 = *reinterpret_cast<const float4*>(&tr.v[8]);
            const float4 b = box[slot];
            touch = b.x <= x1 && b.z >= x0 && b.y <= y1 && b.w >= y0;
        }
        uint64_t m = wave_mask(touch);
        while (m) {
            const int l = __builtin_ctzll(m);
            m &= m - 1;
            if (NP > 1 && (rank_t++ % NP) != part) continue;
            const int s = __builtin_amdgcn_readlane(slot, l);
            auto rl = [l](float x) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l)); };
            const float v0[3] = {rl(q0.x), rl(q0.y), rl(q0.z)};
            const float v1[3] = {rl(q0.w), rl(q1.x), rl(q1.y)};
            const float v2[3] = {rl(q1.z), rl(q1.w), rl(q2.x)};
            const int face = __builtin_amdgcn_readlane(__float_as_int(q2.y), l);
            const float a0 = comp(v0, r.kz), a1 = comp(v1, r.kz), a2 = comp(v2, r.kz);
            const float near = r.Sz > 0.0f ? fminf(fminf(a0, a1), a2) : fmaxf(fmaxf(a0, a1), a2);
            const float bound = r.Sz * (near - okz);
            const bool need = active && !(bound * (1.0f - 1e-6f) > tb);
            if (COUNT && active) { tc->nodes++; tc->nodes_w++; }
            const uint64_t mn = wave_mask(need);
            if (mn == 0) continue;
            if (COUNT) {
                if (need) tc->tris++;
                if (active) tc->tris_w++;
            }
            float t, U, V, W, det;
            if (watertight(r, v0, v1, v2, t, U, V, W, det)) {
                if (t < tb || (t == tb && face < fb)) {
                    tb = t; fb = face;
                    h.face = face;
                    h.slot = s;
                    h.t = t;
                }
            }
        }
    }
}

// float64 direction of the ray through screen point (X, Y)
__device__ __forceinline__ void ray_dir64(const ViewDev& c, double X, double Y, double* d)
{
    double dcx = (X - (double)c.cx) / (double)c.fx;
    double dcy = (Y - (double)c.cy) / (double)c.fy;
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = (double)c.R[k] * dcx + (double)c.R[3 + k] * dcy + (double)c.R[6 + k];
}

// Hard rasterisation (the comparison renderer of Section 4.2.2, "Ray tracing
// vs rasterization"): one sample at the pixel centre, the triangle covering it
// with the largest perspective-correct 1/z wins.  Coverage: the edge functions
// E(a, b, p) = (b.x - a.x)(p.y - a.y) - (b.y - a.y)(p.x - a.x) of the edges
// (v1, v2), (v2, v0), (v0, v1) are all >= 0 or all <= 0 with a non-zero sum
// (no culling; a centre on a shared edge is covered by both triangles);
// triangles with a vertex less than 1 mm in front of the camera are dropped;
// 1/z = (E0/z0 + E1/z1 + E2/z2) / (E0 + E1 + E2), compared rounded to
// float32, ties to the smaller triangle index.  Projection, edge functions and
// 1/z in float64 from the float32 vertices, each expression in one fixed
// order (no contraction), so the covering triangle is reproducible exactly.
constexpr uint64_t kCentreWord = 0x8000000080000000ull;   // sample word with u = v = 1/2
constexpr double kRasterNear = 1e-3;

__device__ __forceinline__ void raster_project(const ViewDev& c, const float v[3], double& px, double& py,
                                               double& z)
{
    const double q0 = (double)v[0] - (double)c.o[0], q1 = (double)v[1] - (double)c.o[1];
    const double q2 = (double)v[2] - (double)c.o[2];
    const double x = ((double)c.R[0] * q0 + (double)c.R[1] * q1) + (double)c.R[2] * q2;
    const double y = ((double)c.R[3] * q0 + (double)c.R[4] * q1) + (double)c.R[5] * q2;
    z = ((double)c.R[6] * q0 + (double)c.R[7] * q1) + (double)c.R[8] * q2;
    px = ((double)c.fx * x) / z + (double)c.cx;
    py = ((double)c.fy * y) / z + (double)c.cy;
}

__device__ __forceinline__ double raster_edge(double ax, double ay, double bx, double by, double px, double py)
{
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

// Covering triangle of pixel centre (X, Y) among `cnt` listed leaf slots
// (`ent`, or slots 0 .. cnt-1 when null; `box` the slots' padded screen bounds
// against the tile rectangle [x0, x1] x [y0, y1], or no bound test when
// null).  The calling lanes load the list together, as trace_bins does.
template <bool COUNT>
__device__ __forceinline__ void raster_list(const Tri* __restrict__ tris, const uint16_t* __restrict__ ent, int cnt,
                                            const float4* __restrict__ box, float x0, float y0, float x1, float y1,
                                            const ViewDev& c, double X, double Y, bool active, Hit& h,
                                            TraceCount* tc = nullptr)
{
    h.face = -1;
    h.slot = 0;
    h.t = 0.0f;
    uint32_t bk = 0u;   // float32 bits of the best 1/z (0: none)
    int bf = 0x7fffffff;
    tris = uniform_ptr(tris);
    const uint64_t exec = wave_mask(true);
    const int ncall = __popcll(exec);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(exec >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)exec, 0u));
    for (int c0 = 0; c0 < cnt; c0 += ncall) {
        int slot = 0;
        bool touch = false;
        float4 q0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), q1 = q0, q2 = q0;
        if (c0 + rank < cnt) {
            slot = ent ? (int)ent[c0 + rank] : c0 + rank;
            const Tri& tr = tris[slot];
            q0 = *reinterpret_cast<const float4*>(&tr.v[0]);
            q1 = *reinterpret_cast<const float4*>(&tr.v[4]);
            q2 = *reinterpret_cast<const float4*>(&tr.v[8]);
            touch = true;
            if (box) {
                const float4 b = box[slot];
                touch = b.x <= x1 && b.z >= x0 && b.y <= y1 && b.w >= y0;
            }
        }
        uint64_t m = wave_mask(touch);
        while (m) {
            const int l = __builtin_ctzll(m);
            m &= m - 1;
            const int s = __builtin_amdgcn_readlane(slot, l);
            auto rl = [l](float x) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l)); };
            const float v0[3] = {rl(q0.x), rl(q0.y), rl(q0.z)};
            const float v1[3] = {rl(q0.w), rl(q1.x), rl(q1.y)};
            const float v2[3] = {rl(q1.z), rl(q1.w), rl(q2.x)};
            const int face = __builtin_amdgcn_readlane(__float_as_int(q2.y), l);
            if (COUNT && active) { tc->nodes++; tc->nodes_w++; tc->tris++; tc->tris_w++; }
            double ax, ay, az, bx, by, bz, cx, cy, cz;
            raster_project(c, v0, ax, ay, az);
            raster_project(c, v1, bx, by, bz);
            raster_project(c, v2, cx, cy, cz);
            if (!(az > kRasterNear && bz > kRasterNear && cz > kRasterNear)) continue;   // uniform
            const double e0 = raster_edge(bx, by, cx, cy, X, Y);
            const double e1 = raster_edge(cx, cy, ax, ay, X, Y);
            const double e2 = raster_edge(ax, ay, bx, by, X, Y);
            const double area = (e0 + e1) + e2;
            const bool in = ((e0 >= 0.0 && e1 >= 0.0 && e2 >= 0.0) || (e0 <= 0.0 && e1 <= 0.0 && e2 <= 0.0)) &&
                            area != 0.0;
            if (!(active && in)) continue;
            const double zinv = ((e0 / az + e1 / bz) + e2 / cz) / area;
            const uint32_t key = __float_as_uint((float)zinv);
            if (key > bk || (key == bk && face < bf)) {
                bk = key;
                bf = face;
                h.face = face;
                h.slot = s;
            }
        }
    }
}

// barycentrics of the hit on triangle `slot` for the float64 ray (o, d):
// o + t d = (1-b1-b2) v0 + b1 v1 + b2 v2 by Cramer's rule
__device__ __forceinline__ void surface(const Tri* __restrict__ tris, const float* __restrict__ uv, int slot,
                                        const ViewDev& c, double X, double Y, Surf& s)
{
    const Tri& tr = tris[slot];
    float4 p0 = *reinterpret_cast<const float4*>(&tr.v[0]);
    float4 p1 = *reinterpret_cast<const float4*>(&tr.v[4]);
    float4 p2 = *reinterpret_cast<const float4*>(&tr.v[8]);
    s.v[0] = p0.x; s.v[1] = p0.y; s.v[2] = p0.z; s.v[3] = p0.w; s.v[4] = p1.x;
    s.v[5] = p1.y; s.v[6] = p1.z; s.v[7] = p1.w; s.v[8] = p2.x;
    s.face = __float_as_int(p2.y);
    s.i0 = __float_as_int(p2.z); s.i1 = __float_as_int(p2.w); s.i2 = tr.i2;
    ray_dir64(c, X, Y, s.d);
    double e1[3], e2[3], q[3], pv[3], sv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e1[k] = (double)s.v[3 + k] - (double)s.v[k];
        e2[k] = (double)s.v[6 + k] - (double)s.v[k];
        sv[k] = (double)c.o[k] - (double)s.v[k];
    }
    pv[0] = s.d[1] * e2[2] - s.d[2] * e2[1];
    pv[1] = s.d[2] * e2[0] - s.d[0] * e2[2];
    pv[2] = s.d[0] * e2[1] - s.d[1] * e2[0];
    double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    q[0] = sv[1] * e1[2] - sv[2] * e1[1];
    q[1] = sv[2] * e1[0] - sv[0] * e1[2];
    q[2] = sv[0] * e1[1] - sv[1] * e1[0];
    const double idet = 1.0 / det;
    double b1 = (sv[0] * pv[0] + sv[1] * pv[1] + sv[2] * pv[2]) * idet;
    double b2 = (s.d[0] * q[0] + s.d[1] * q[1] + s.d[2] * q[2]) * idet;
    s.idet = idet;
    s.pv[0] = pv[0]; s.pv[1] = pv[1]; s.pv[2] = pv[2];
    const double b0 = 1.0 - b1 - b2;
    s.b0 = (float)b0;
    s.b1 = (float)b1;
    s.b2 = (float)b2;
    const float2 uv0 = *reinterpret_cast<const float2*>(uv + 2 * s.i0);
    const float2 uv1 = *reinterpret_cast<const float2*>(uv + 2 * s.i1);
    const float2 uv2 = *reinterpret_cast<const float2*>(uv + 2 * s.i2);
    s.tu = b0 * (double)uv0.x + b1 * (double)uv1.x + b2 * (double)uv2.x;
    s.tv = b0 * (double)uv0.y + b1 * (double)uv1.y + b2 * (double)uv2.y;
}

// ---------------------------------------------------------------------------
// shading: albedo(uv) * (ka + kd max(0, n.l)), bilinear albedo with texel
// centres at (j + 1/2) / W, clamped at the border
// ---------------------------------------------------------------------------

struct Shading {
    float ka, kd, l[3];
};

struct Shade {
    float u, v;                 // texture coordinates
    float n[3], nlen;           // unit interpolated normal and the raw length
    float ndotl, shade;
    int idx[4];                 // texel indices
    int ti0, ti1, tj0, tj1;     // texel rows / columns of the bilinear footprint
    float w[4];                 // bilinear weights
    float col[3];               // albedo
    float dcol_du[3], dcol_dv[3];
};

__device__ __forceinline__ void shade_hit(const Surf& h, const float* __restrict__ normals,
                                          const float* __restrict__ uv, const float* __restrict__ tex,
                                          int th, int tw, const Shading& S, Shade& o)
{
    const float b0 = h.b0, b1 = h.b1, b2 = h.b2;
    o.u = (float)h.tu;
    o.v = (float)h.tv;
    const float* n0 = normals + 3 * h.i0;
    const float* n1 = normals + 3 * h.i1;
    const float* n2 = normals + 3 * h.i2;
    float nr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) nr[k] = b0 * n0[k] + b1 * n1[k] + b2 * n2[k];
    o.nlen = sqrtf(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
    float inl = 1.0f / o.nlen;
#pragma unroll
    for (int k = 0; k < 3; ++k) o.n[k] = nr[k] * inl;
    o.ndotl = o.n[0] * S.l[0] + o.n[1] * S.l[1] + o.n[2] * S.l[2];
    o.shade = S.ka + S.kd * fmaxf(o.ndotl, 0.0f);
    const double x = h.tu * tw - 0.5, y = h.tv * th - 0.5;
    const double fx0 = floor(x), fy0 = floor(y);
    const float ax = (float)(x - fx0), ay = (float)(y - fy0);
    int j0 = (int)fx0, i0 = (int)fy0;
    int j1 = min(max(j0 + 1, 0), tw - 1), i1 = min(max(i0 + 1, 0), th - 1);
    j0 = min(max(j0, 0), tw - 1);
    i0 = min(max(i0, 0), th - 1);
    o.ti0 = i0; o.ti1 = i1; o.tj0 = j0; o.tj1 = j1;
    o.idx[0] = i0 * tw + j0; o.w[0] = (1.0f - ax) * (1.0f - ay);
    o.idx[1] = i0 * tw + j1; o.w[1] = ax * (1.0f - ay);
    o.idx[2] = i1 * tw + j0; o.w[2] = (1.0f - ax) * ay;
    o.idx[3] = i1 * tw + j1; o.w[3] = ax * ay;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float a00 = tex[3 * o.idx[0] + ch], a01 = tex[3 * o.idx[1] + ch];
        float a10 = tex[3 * o.idx[2] + ch], a11 = tex[3 * o.idx[3] + ch];
        o.col[ch] = o.w[0] * a00 + o.w[1] * a01 + o.w[2] * a10 + o.w[3] * a11;
        o.dcol_du[ch] = tw * ((1.0f - ay) * (a01 - a00) + ay * (a11 - a10));
        o.dcol_dv[ch] = th * ((1.0f - ax) * (a10 - a00) + ax * (a11 - a01));
    }
}

// ---------------------------------------------------------------------------
// float32 projection (edge decisions)
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool project32(const ViewDev& c, const float* v, float& px, float& py)
{
    float q0 = v[0] - c.o[0], q1 = v[1] - c.o[1], q2 = v[2] - c.o[2];
    float xc = (c.R[0] * q0 + c.R[1] * q1) + c.R[2] * q2;
    float yc = (c.R[3] * q0 + c.R[4] * q1) + c.R[5] * q2;
    float zc = (c.R[6] * q0 + c.R[7] * q1) + c.R[8] * q2;
    if (!(zc > 1e-4f)) return false;
    px = (c.fx * xc) / zc + c.cx;
    py = (c.fy * yc) / zc + c.cy;
    return true;
}

// ---------------------------------------------------------------------------
// wave / block reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// The same reductions on the DPP network (lane moves inside the VALU, no LDS
// traffic).  DPP rows are groups of 16 lanes; update_dpp with old = 0 and
// bound_ctrl set reads 0 where the source lane is outside the row, and keeps
// 0 in rows the row mask leaves out.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

// sum over the 64 lanes, complete in lane 63: prefix sums inside each row
// (shifts by 1, 2, 4, 8), then lane 15 into rows 1 and 3 and lane 31 into
// rows 2 and 3
__device__ __forceinline__ float wave_sum63(float v)
{
    v += dpp_f<0x111>(v);
    v += dpp_f<0x112>(v);
    v += dpp_f<0x114>(v);
    v += dpp_f<0x118>(v);
    v += dpp_f<0x142, 0xA>(v);
    v += dpp_f<0x143, 0xC>(v);
    return v;
}

// wave_sum63 of N values at once, step by step over all of them (the DPP
// steps of different values interleave instead of waiting on each other)
template <int N>
__device__ __forceinline__ void wave_sum63_n(float* v)
{
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_f<0x111>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_f<0x112>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_f<0x114>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_f<0x118>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_f<0x142, 0xA>(v[k]);
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_f<0x143, 0xC>(v[k]);
}

// min / max over each row of 16 lanes, in every lane of the row: swaps inside
// quads (lane ^ 1, lane ^ 2), then the half-row and row mirrors
__device__ __forceinline__ int row_min(int v)
{
    v = min(v, dpp_i<0xB1>(v));
    v = min(v, dpp_i<0x4E>(v));
    v = min(v, dpp_i<0x141>(v));
    v = min(v, dpp_i<0x140>(v));
    return v;
}

__device__ __forceinline__ int row_max(int v)
{
    v = max(v, dpp_i<0xB1>(v));
    v = max(v, dpp_i<0x4E>(v));
    v = max(v, dpp_i<0x141>(v));
    v = max(v, dpp_i<0x140>(v));
    return v;
}

// order the wave's LDS accesses across lanes (no block barrier: waves of a
// block run independently in the persistent loops)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Block-wide copy of n elements from global memory into LDS, eight loads in
// flight per thread (a staging loop that waits on each load in turn costs a
// memory round trip per element and thread).  The caller synchronises.
template <typename T>
__device__ __forceinline__ void lds_stage(T* dst, const T* __restrict__ src, int n)
{
    const int s = blockDim.x;
    int i = threadIdx.x;
    for (; i + 7 * s < n; i += 8 * s) {
        T r[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) r[k] = src[i + k * s];
#pragma unroll
        for (int k = 0; k < 8; ++k) dst[i + k * s] = r[k];
    }
    T r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (i + k * s < n) r[k] = src[i + k * s];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (i + k * s < n) dst[i + k * s] = r[k];
}

}  // namespace hr
