// handrt kernels for gfx950: skinning, geometry preparation (vertex normals,
// bounding-volume refit, per-view screen bounds), rendering, L1 loss, interior
// adjoint, silhouette edges and edge sampling, normals + skinning backward, Adam.
#include "kernels.h"

namespace hr {

// ===========================================================================
// skinning (forward)
// ===========================================================================

struct Rod {                  // R = I + a K + b K^2 and the derivative factors
    float R[9];
    float a, b, ad, bd;       // ad = a'(|r|)/|r|, bd = b'(|r|)/|r|
};

__device__ void rodrigues(const float* r, Rod& o)
{
    float t2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    float t = sqrtf(t2);
    if (t < 0.3f) {
        // series (no cancellation for small angles)
        o.a = 1.0f - t2 / 6.0f + t2 * t2 / 120.0f;
        o.b = 0.5f - t2 / 24.0f + t2 * t2 / 720.0f;
        o.ad = -1.0f / 3.0f + t2 / 30.0f - t2 * t2 / 840.0f;
        o.bd = -1.0f / 12.0f + t2 / 180.0f - t2 * t2 / 6720.0f;
    } else {
        float s = sinf(t), c = cosf(t), sh = sinf(0.5f * t);
        o.a = s / t;
        o.b = 2.0f * sh * sh / t2;
        o.ad = (t * c - s) / (t2 * t);
        o.bd = (t * s - 4.0f * sh * sh) / (t2 * t2);
    }
    float K[9] = {0.0f, -r[2], r[1], r[2], 0.0f, -r[0], -r[1], r[0], 0.0f};
    float K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K2[3 * i + j] = K[3 * i + 0] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    for (int i = 0; i < 9; ++i) o.R[i] = o.a * K[i] + o.b * K2[i];
    o.R[0] += 1.0f; o.R[4] += 1.0f; o.R[8] += 1.0f;
}

// <G, K(e_k)> for k = 0..2, K(e) the cross-product matrix of e
__device__ __forceinline__ void skew_dot(const float* G, float* out)
{
    out[0] = G[7] - G[5];
    out[1] = G[2] - G[6];
    out[2] = G[3] - G[1];
}

// gradient of <gR, R(r)> with respect to r
__device__ void rodrigues_bwd(const float* r, const Rod& d, const float* gR, float* gr)
{
    float K[9] = {0.0f, -r[2], r[1], r[2], 0.0f, -r[0], -r[1], r[0], 0.0f};
    float K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K2[3 * i + j] = K[3 * i + 0] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    float gK = 0.0f, gK2 = 0.0f;
    for (int i = 0; i < 9; ++i) { gK += gR[i] * K[i]; gK2 += gR[i] * K2[i]; }
    // X = gR K^T + K^T gR: <gR, E K + K E> = <X, E>
    float X[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            float s = 0.0f;
            for (int m = 0; m < 3; ++m) s += gR[3 * i + m] * K[3 * j + m] + K[3 * m + i] * gR[3 * m + j];
            X[3 * i + j] = s;
        }
    float s1[3], s2[3];
    skew_dot(gR, s1);
    skew_dot(X, s2);
    for (int k = 0; k < 3; ++k) gr[k] = d.ad * r[k] * gK + d.a * s1[k] + d.bd * r[k] * gK2 + d.b * s2[k];
}

__device__ __forceinline__ void matmul3(const float* A, const float* B, float* C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

__device__ __forceinline__ void matvec3(const float* A, const float* x, float* y)
{
    for (int i = 0; i < 3; ++i) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}

__device__ __forceinline__ void matTvec3(const float* A, const float* x, float* y)
{
    for (int i = 0; i < 3; ++i) y[i] = A[i] * x[0] + A[3 + i] * x[1] + A[6 + i] * x[2];
}

// Joint transforms of one hand, in LDS (computed by every block that needs
// them: a few hundred flops against the latency of a second launch).
struct JointState {
    Rod rod[kMaxJoints + 1];      // joint rotations and the global rotation
    float GR[kMaxJoints * 9];     // world rotation of each joint frame
    float Gt[kMaxJoints * 3];     // world position of each joint
    float At[kMaxJoints * 3];     // Gt - GR J: translation of the skinning transform
    float J[kMaxJoints * 3];      // rest joint positions (shaped)
    float Rp[9];                  // global rotation
};
constexpr int kJointStateFloats = sizeof(JointState) / sizeof(float);

// Small per-vertex and per-joint tables are read into registers with loads
// that do not depend on a branch (indices clamped into range, the surplus
// entries zeroed afterwards), so each group is one round trip to memory
// instead of one per entry.

// shape coefficients, zero beyond K
__device__ __forceinline__ void load_beta(const MeshDev& m, const float* __restrict__ beta, float* bk)
{
    const int K = m.K;
#pragma unroll
    for (int k = 0; k < kMaxShape; ++k) {
        const float b = K > 0 ? beta[k < K ? k : K - 1] : 0.0f;
        bk[k] = k < K ? b : 0.0f;
    }
}

// skinning weights of vertex v (wq = 0 beyond m.infl <= kMaxInfl)
__device__ __forceinline__ void load_weights(const MeshDev& m, int v, float* wq, int* jq)
{
    const int n = m.infl;
#pragma unroll
    for (int q = 0; q < kMaxInfl; ++q) {
        const int qq = q < n ? q : n - 1;
        const float w = m.wval[(size_t)qq * m.V + v];
        jq[q] = m.widx[(size_t)qq * m.V + v];
        wq[q] = q < n ? w : 0.0f;
    }
}

// Rodrigues rotations, joint positions J = J_reg T + (J_reg S) beta (the
// regressor applied to the template and the shape directions once, at scene
// creation), forward kinematics one tree level at a time.  The first wave
// does the work (J < 64: the levels synchronise the wave only); every
// thread of the block must call it (it ends with a block barrier).
__device__ void joint_state(const MeshDev& m, const float* __restrict__ p, JointState& js)
{
    const int J = m.J, K = m.K;
    const int j = threadIdx.x;
    if (j < 64) {
        // every load first (the LDS stores below could alias them otherwise)
        float bk[kMaxShape];
        load_beta(m, p + 48, bk);
        const int dj = j < J ? m.jdepth[j] : -1, par = j < J ? m.parents[j] : -1;
        const int jr = j < J ? j : J;
        const float* pr = j < J ? p + 3 * j : p + 58;
        const float r[3] = {pr[0], pr[1], pr[2]};
        const int jj = j < J ? j : J - 1;
        float jt[3], jsd[3][kMaxShape];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            jt[c] = m.jt[3 * jj + c];
#pragma unroll
            for (int k = 0; k < kMaxShape; ++k) {
                const float d = K > 0 ? m.js[(3 * jj + c) * K + (k < K ? k : K - 1)] : 0.0f;
                jsd[c][k] = k < K ? d : 0.0f;
            }
        }
        if (j <= J) rodrigues(r, js.rod[jr]);
        if (j < J)
            for (int c = 0; c < 3; ++c) {
                float x = jt[c];
#pragma unroll
                for (int k = 0; k < kMaxShape; ++k)
                    if (k < K) x += jsd[c][k] * bk[k];
                js.J[3 * j + c] = x;
            }
        wave_lds_sync();
        if (j < 9) js.Rp[j] = js.rod[J].R[j];
        for (int L = 0; L <= m.max_depth; ++L) {
            if (dj == L) {
                if (par < 0) {
                    for (int i = 0; i < 9; ++i) js.GR[9 * j + i] = js.rod[j].R[i];
                    for (int i = 0; i < 3; ++i) js.Gt[3 * j + i] = js.J[3 * j + i];
                } else {
                    matmul3(js.GR + 9 * par, js.rod[j].R, js.GR + 9 * j);
                    float d[3] = {js.J[3 * j] - js.J[3 * par], js.J[3 * j + 1] - js.J[3 * par + 1],
                                  js.J[3 * j + 2] - js.J[3 * par + 2]};
                    float y[3];
                    matvec3(js.GR + 9 * par, d, y);
                    for (int i = 0; i < 3; ++i) js.Gt[3 * j + i] = y[i] + js.Gt[3 * par + i];
                }
                float y[3];
                matvec3(js.GR + 9 * j, js.J + 3 * j, y);
                for (int i = 0; i < 3; ++i) js.At[3 * j + i] = js.Gt[3 * j + i] - y[i];
            }
            wave_lds_sync();
        }
    }
    __syncthreads();
}

// shaped vertex v: T_v + S_v beta (bk from load_beta)
// the vertex's rest data: template position and shape directions (sd
// entries past K repeat entry K - 1)
__device__ __forceinline__ void load_shape(const MeshDev& m, int v, float* tpl, float (&sd)[3][kMaxShape])
{
    const int K = m.K;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        tpl[c] = m.v_template[(size_t)c * m.V + v];
#pragma unroll
        for (int k = 0; k < kMaxShape; ++k)
            sd[c][k] = K > 0 ? m.shapedirs[((size_t)(k < K ? k : K - 1) * 3 + c) * m.V + v] : 0.0f;
    }
}

__device__ __forceinline__ void shape_vertex(const MeshDev& m, const float* bk, const float* tpl,
                                             const float (&sd)[3][kMaxShape], float* x)
{
    const int K = m.K;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float s = tpl[c];
#pragma unroll
        for (int k = 0; k < kMaxShape; ++k)
            if (k < K) s += sd[c][k] * bk[k];
        x[c] = s;
    }
}

__device__ __forceinline__ void shaped_vertex(const MeshDev& m, const float* bk, int v, float* x,
                                              float (&sd)[3][kMaxShape])
{
    float tpl[3];
    load_shape(m, v, tpl, sd);
    shape_vertex(m, bk, tpl, sd, x);
}

// posed (pre-global-transform) vertex: sum over the vertex's skinning
// weights (from load_weights)
__device__ __forceinline__ void blend_vertex(const JointState& js, const float* wq, const int* jq, const float* x,
                                             float* vp)
{
    vp[0] = vp[1] = vp[2] = 0.0f;
#pragma unroll
    for (int q = 0; q < kMaxInfl; ++q) {
        const float w = wq[q];
        if (w == 0.0f) continue;
        const int j = jq[q];
        float y[3];
        matvec3(js.GR + 9 * j, x, y);
        for (int c = 0; c < 3; ++c) vp[c] += w * (y[c] + js.At[3 * j + c]);
    }
}

__device__ __forceinline__ void shaped_vertex(const MeshDev& m, const float* bk, int v, float* x)
{
    float sd[3][kMaxShape];
    shaped_vertex(m, bk, v, x, sd);
}

// ---------------------------------------------------------------------------
// Forward skinning in float64.  The model's real tables hold float32 values,
// whose float64 conversions are exact, so the vertices are the float32
// roundings of a float64 evaluation of the skinning: the same float32 values
// a float64 evaluation elsewhere rounds to (bar ties), which keeps every
// float32 decision downstream (hits, silhouettes) identical.  The joint state
// handed to the float32 backward is the rounding of the float64 one.
// ---------------------------------------------------------------------------

struct Rod64 {
    double R[9];
    double a, b, ad, bd;
};

struct JointState64 {              // JointState's layout with float64 members
    Rod64 rod[kMaxJoints + 1];
    double GR[kMaxJoints * 9];
    double Gt[kMaxJoints * 3];
    double At[kMaxJoints * 3];
    double J[kMaxJoints * 3];
    double Rp[9];
};
static_assert(sizeof(JointState64) == 2 * sizeof(JointState), "joint state layouts differ");

__device__ void rodrigues64(const double* r, Rod64& o)
{
    const double t2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double t = sqrt(t2);
    // the three circular functions once, for every lane: the lanes of a wave
    // take different branches below, which would otherwise each evaluate them
    const double s = sin(t), c = cos(t), sh = sin(0.5 * t);
    if (t < 1e-4) {
        o.a = 1.0 - t2 / 6.0;
        o.b = 0.5 - t2 / 24.0;
    } else {
        o.a = s / t;
        o.b = 2.0 * sh * sh / t2;
    }
    // derivative factors of the backward (float32 there)
    if (t < 0.3) {
        o.ad = -1.0 / 3.0 + t2 / 30.0 - t2 * t2 / 840.0;
        o.bd = -1.0 / 12.0 + t2 / 180.0 - t2 * t2 / 6720.0;
    } else {
        o.ad = (t * c - s) / (t2 * t);
        o.bd = (t * s - 4.0 * sh * sh) / (t2 * t2);
    }
    const double K[9] = {0.0, -r[2], r[1], r[2], 0.0, -r[0], -r[1], r[0], 0.0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double k2 = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
            o.R[3 * i + j] = o.a * K[3 * i + j] + o.b * k2 + (i == j ? 1.0 : 0.0);
        }
}

__device__ __forceinline__ void matmul3d(const double* A, const double* B, double* C)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

__device__ __forceinline__ void matvec3d(const double* A, const double* x, double* y)
{
    for (int i = 0; i < 3; ++i) y[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
}

// joint_state in float64, in the first wave: lane j < J for joint j, lane J
// for the global rotation.  The tree is walked one level at a time from the
// roots with each lane's global rotation and translation in registers: a
// lane of level L reads its parent's (final since level L - 1) from the
// parent's lane, so no level waits on LDS.  The products are those of
// joint_state, in the same order.  Ends with a block barrier.
__device__ void joint_state64(const MeshDev& m, const float* __restrict__ p, JointState64& js)
{
    const int J = m.J, K = m.K;
    const int j = threadIdx.x;
    if (j < 64) {
        // every load first, with clamped indices (one round trip to memory)
        float bkf[kMaxShape];
        load_beta(m, p + 48, bkf);
        const int dj = j < J ? m.jdepth[j] : -1, par = j < J ? m.parents[j] : -1;
        const int jr = j < J ? j : J;
        const float* pr = j < J ? p + 3 * j : p + 58;
        const double r[3] = {(double)pr[0], (double)pr[1], (double)pr[2]};
        const int jj = j < J ? j : J - 1;
        double jt[3], jsd[3][kMaxShape];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            jt[c] = m.jt64[3 * jj + c];
#pragma unroll
            for (int k = 0; k < kMaxShape; ++k) {
                const double d = K > 0 ? m.js64[(3 * jj + c) * K + (k < K ? k : K - 1)] : 0.0;
                jsd[c][k] = k < K ? d : 0.0;
            }
        }
        Rod64 rd;
        rodrigues64(r, rd);
        if (j <= J) js.rod[jr] = rd;
        if (j == J)
            for (int i = 0; i < 9; ++i) js.Rp[i] = rd.R[i];
        double x[3];
        for (int c = 0; c < 3; ++c) {
            x[c] = jt[c];
#pragma unroll
            for (int k = 0; k < kMaxShape; ++k)
                if (k < K) x[c] += jsd[c][k] * (double)bkf[k];
        }
        if (j < J)
            for (int c = 0; c < 3; ++c) js.J[3 * j + c] = x[c];
        // roots: GR = R, Gt = J; lane `src` is the parent (itself for roots
        // and lanes past the joints)
        const int src = par >= 0 ? par : j;
        double GR[9], Gt[3], pJ[3];
        for (int i = 0; i < 9; ++i) GR[i] = rd.R[i];
        for (int c = 0; c < 3; ++c) {
            Gt[c] = x[c];
            pJ[c] = __shfl(x[c], src);
        }
        for (int L = 1; L <= m.max_depth; ++L) {
            double pG[9], pt[3];
            for (int i = 0; i < 9; ++i) pG[i] = __shfl(GR[i], src);
            for (int i = 0; i < 3; ++i) pt[i] = __shfl(Gt[i], src);
            if (dj == L) {
                matmul3d(pG, rd.R, GR);
                const double d[3] = {x[0] - pJ[0], x[1] - pJ[1], x[2] - pJ[2]};
                double y[3];
                matvec3d(pG, d, y);
                for (int i = 0; i < 3; ++i) Gt[i] = y[i] + pt[i];
            }
        }
        if (j < J) {
            double y[3];
            matvec3d(GR, x, y);
            for (int i = 0; i < 9; ++i) js.GR[9 * j + i] = GR[i];
            for (int i = 0; i < 3; ++i) {
                js.Gt[3 * j + i] = Gt[i];
                js.At[3 * j + i] = Gt[i] - y[i];
            }
        }
    }
    __syncthreads();
}

// Skinning, grid (vertex blocks, hands).
__global__ void __launch_bounds__(128) k_skin(MeshDev m, const float* __restrict__ params,
                                              float* __restrict__ verts, float* __restrict__ joints,
                                              int* __restrict__ tile_count, float* __restrict__ js_out)
{
    __shared__ JointState64 js;
    const int h = blockIdx.y;
    // nullable: the wave-tile list of a following refit starts empty
    if (tile_count && blockIdx.x == 0 && h == 0 && threadIdx.x == 0) *tile_count = 0;
    const float* p = params + 64 * h;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    // the vertex's tables first: their loads are in flight with the joint
    // state's
    float tpl[3] = {0.0f, 0.0f, 0.0f}, sd[3][kMaxShape] = {}, wq[kMaxInfl] = {}, bk[kMaxShape];
    int jq[kMaxInfl] = {};
    if (v < m.V) {
        load_weights(m, v, wq, jq);
        load_shape(m, v, tpl, sd);
    }
    load_beta(m, p + 48, bk);
    const float tau[3] = {p[61], p[62], p[63]};
    joint_state64(m, p, js);
    // nullable: the joint state of these parameters for the backward (float32)
    if (js_out && blockIdx.x == 0) {
        const double* src = reinterpret_cast<const double*>(&js);
        for (int i = threadIdx.x; i < kJointStateFloats; i += blockDim.x)
            js_out[(size_t)h * kJointStateFloats + i] = (float)src[i];
    }
    if (v < m.V) {
        double x[3], vp[3] = {0.0, 0.0, 0.0}, y[3];
        for (int c = 0; c < 3; ++c) {
            double sv = (double)tpl[c];
#pragma unroll
            for (int k = 0; k < kMaxShape; ++k)
                if (k < m.K) sv += (double)sd[c][k] * (double)bk[k];
            x[c] = sv;
        }
#pragma unroll
        for (int q = 0; q < kMaxInfl; ++q) {
            const double w = (double)wq[q];
            if (w == 0.0) continue;
            const int j = jq[q];
            double g[3];
            matvec3d(js.GR + 9 * j, x, g);
            for (int c = 0; c < 3; ++c) vp[c] += w * (g[c] + js.At[3 * j + c]);
        }
        matvec3d(js.Rp, vp, y);
        float* o = verts + ((size_t)h * m.V + v) * 3;
        o[0] = (float)(y[0] + (double)tau[0]);
        o[1] = (float)(y[1] + (double)tau[1]);
        o[2] = (float)(y[2] + (double)tau[2]);
    }
    if (joints && blockIdx.x == 0 && (int)threadIdx.x < m.J) {
        const int j = threadIdx.x;
        double y[3];
        matvec3d(js.Rp, js.Gt + 3 * j, y);
        float* o = joints + ((size_t)h * m.J + j) * 3;
        o[0] = (float)(y[0] + (double)tau[0]);
        o[1] = (float)(y[1] + (double)tau[1]);
        o[2] = (float)(y[2] + (double)tau[2]);
    }
}

// ===========================================================================
// geometry preparation: vertex normals, triangles in leaf order, BVH refit
// ===========================================================================

__device__ void normals_hand(const MeshDev& m, const float* __restrict__ verts, float* __restrict__ normals, int h,
                             float* dyn)
{
    const int V = m.V, F = m.F;
    float* vsh = dyn;          // [V*3]
    float* fn = vsh + 3 * V;   // [F*3] raw face normals (area weighted)
    lds_stage(vsh, verts + (size_t)h * V * 3, 3 * V);
    __syncthreads();
    for (int f = threadIdx.x; f < F; f += blockDim.x) {
        int a = m.faces[3 * f], bb = m.faces[3 * f + 1], c = m.faces[3 * f + 2];
        float e1[3] = {vsh[3 * bb] - vsh[3 * a], vsh[3 * bb + 1] - vsh[3 * a + 1], vsh[3 * bb + 2] - vsh[3 * a + 2]};
        float e2[3] = {vsh[3 * c] - vsh[3 * a], vsh[3 * c + 1] - vsh[3 * a + 1], vsh[3 * c + 2] - vsh[3 * a + 2]};
        fn[3 * f] = e1[1] * e2[2] - e1[2] * e2[1];
        fn[3 * f + 1] = e1[2] * e2[0] - e1[0] * e2[2];
        fn[3 * f + 2] = e1[0] * e2[1] - e1[1] * e2[0];
    }
    __syncthreads();
    float* nh = normals + (size_t)h * V * 3;
    for (int v = threadIdx.x; v < V; v += blockDim.x) {
        float s[3] = {0.0f, 0.0f, 0.0f};
        for (int k = m.vf_off[v]; k < m.vf_off[v + 1]; ++k) {
            int f = m.vf_faces[k];
            s[0] += fn[3 * f]; s[1] += fn[3 * f + 1]; s[2] += fn[3 * f + 2];
        }
        float inv = 1.0f / sqrtf(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        nh[3 * v] = s[0] * inv; nh[3 * v + 1] = s[1] * inv; nh[3 * v + 2] = s[2] * inv;
    }
}

__device__ __forceinline__ float box_area(const float* lo, const float* hi)
{
    const float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return 2.0f * (dx * dy + dy * dz + dz * dx);
}

// Refit of hand h's hierarchy; with cost, also its quality: the sum over
// the internal nodes of their two child boxes' surface areas over the root
// box's (the expected number of child-box tests of a ray through the root
// box, the surface-area measure a topology build minimises).  It grows as
// the pose drifts from the one the topology was built for.
__device__ void refit_hand(const MeshDev& m, const BvhDev& b, const float* __restrict__ verts,
                           Tri* __restrict__ tris, Node* __restrict__ nodes, int h, float* dyn,
                           float* __restrict__ cost)
{
    const int V = m.V, F = m.F, NS = b.node_stride;
    // LDS: vertices, node bounds, child codes, vertex ids of the leaf slots,
    // each slot's triangle bounds, the level offsets: every refit level reads
    // LDS only (a global load in the level loop would also wait for the
    // previous level's node stores)
    float* vsh = dyn;                                        // [V*3]
    float* nb = vsh + 3 * V;                                 // [NS*6] node bounds
    float* sb = nb + 6 * NS;                                 // [F*6] slot bounds
    int* lchild = reinterpret_cast<int*>(sb + 6 * F);        // [NS*2]
    int* lsv = lchild + 2 * NS;                              // [F*3]
    int* loff = lsv + 3 * F;                                 // [level_stride]
    const int n_levels = b.n_levels[h];
    lds_stage(vsh, verts + (size_t)h * V * 3, 3 * V);
    lds_stage(lchild, b.child + (size_t)h * NS * 2, 2 * NS);
    lds_stage(lsv, b.slot_verts + (size_t)h * F * 3, 3 * F);
    lds_stage(loff, b.level_off + (size_t)h * b.level_stride, b.level_stride);
    __syncthreads();
    const int n_nodes = loff[n_levels];
    // triangles in leaf order (their face and vertex ids are written with
    // the topology) and their bounds
    Tri* th = tris + (size_t)h * F;
    for (int i = threadIdx.x; i < F; i += blockDim.x) {
        const int i0 = lsv[3 * i], i1 = lsv[3 * i + 1], i2 = lsv[3 * i + 2];
        const float v[9] = {vsh[3 * i0], vsh[3 * i0 + 1], vsh[3 * i0 + 2], vsh[3 * i1], vsh[3 * i1 + 1],
                            vsh[3 * i1 + 2], vsh[3 * i2], vsh[3 * i2 + 1], vsh[3 * i2 + 2]};
        float4* dst = reinterpret_cast<float4*>(th + i);
        dst[0] = make_float4(v[0], v[1], v[2], v[3]);
        dst[1] = make_float4(v[4], v[5], v[6], v[7]);
        reinterpret_cast<float*>(dst + 2)[0] = v[8];
        for (int c = 0; c < 3; ++c) {
            sb[6 * i + c] = fminf(fminf(v[c], v[3 + c]), v[6 + c]);
            sb[6 * i + 3 + c] = fmaxf(fmaxf(v[c], v[3 + c]), v[6 + c]);
        }
    }
    __syncthreads();
    // leaf bounds: the union of the leaf's slots, padded, written over the
    // bounds of its first slot (the leaves' slot ranges are disjoint)
    for (int i = threadIdx.x; i < 2 * n_nodes; i += blockDim.x) {
        const int code = lchild[i];
        if (code >= 0) continue;
        const int lc = ~code, start = lc >> 3, cnt = lc & 7;
        float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
#pragma unroll
        for (int j = 0; j < kLeafMax; ++j) {
            if (j < cnt) {
                for (int k = 0; k < 3; ++k) {
                    lo[k] = fminf(lo[k], sb[6 * (start + j) + k]);
                    hi[k] = fmaxf(hi[k], sb[6 * (start + j) + 3 + k]);
                }
            }
        }
        // conservative padding: the float32 watertight test accepts rays a
        // few ulps outside the exact triangle
        for (int k = 0; k < 3; ++k) {
            const float pad = 1e-5f + 1e-6f * fmaxf(fabsf(lo[k]), fabsf(hi[k]));
            sb[6 * start + k] = lo[k] - pad;
            sb[6 * start + 3 + k] = hi[k] + pad;
        }
    }
    __syncthreads();
    // refit, level by level from the leaves up; the nodes at position q of
    // the height order are numbered n_nodes - 1 - q
    Node* nd = nodes + (size_t)h * NS;
    float area = 0.0f;   // this thread's nodes' child-box areas
    for (int L = 0; L < n_levels; ++L) {
        for (int q = loff[L] + threadIdx.x; q < loff[L + 1]; q += blockDim.x) {
            const int n = n_nodes - 1 - q;
            const int c0 = lchild[2 * n], c1 = lchild[2 * n + 1];
            const float* b0 = c0 >= 0 ? nb + 6 * c0 : sb + 6 * ((~c0) >> 3);
            const float* b1 = c1 >= 0 ? nb + 6 * c1 : sb + 6 * ((~c1) >> 3);
            Node out;
            for (int k = 0; k < 3; ++k) {
                out.lo0[k] = b0[k]; out.hi0[k] = b0[3 + k];
                out.lo1[k] = b1[k]; out.hi1[k] = b1[3 + k];
            }
            out.child[0] = c0; out.child[1] = c1;
            out.pad[0] = out.pad[1] = 0;
            nd[n] = out;
            for (int k = 0; k < 3; ++k) {
                nb[6 * n + k] = fminf(out.lo0[k], out.lo1[k]);
                nb[6 * n + 3 + k] = fmaxf(out.hi0[k], out.hi1[k]);
            }
            if (cost) area += box_area(out.lo0, out.hi0) + box_area(out.lo1, out.hi1);
        }
        __syncthreads();
    }
    if (!cost) return;
    // block sum: waves, then the first thread (the root's box is node 0's)
    __shared__ float wsum[16];
    area = wave_sum(area);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = area;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.0f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += wsum[w];
        const float ra = n_nodes > 0 ? box_area(nb, nb + 3) : 0.0f;
        cost[h] = ra > 0.0f ? tot / ra : 0.0f;
    }
}

// Per-view screen bounds of the projected hand, turned into a list of wave
// tiles (tw x th pixels, all samples of a pixel in one wave) appended to
// `tiles` (order across views is arbitrary).  The whole view is listed if any
// vertex is not in front of the camera.
__device__ void view_bounds(const MeshDev& m, const ViewDev* __restrict__ views, const float* __restrict__ verts,
                            TileShape ts, int2* __restrict__ tiles, int* __restrict__ tile_count,
                            int4* __restrict__ view_rect, int vi)
{
    __shared__ float red[4 * 16];
    __shared__ int base;
    const ViewDev c = views[vi];
    const float* vh = verts + (size_t)c.hand * m.V * 3;
    float mnx = 3e38f, mny = 3e38f, mxx = -3e38f, mxy = -3e38f;
    int bad = 0;
    for (int v = threadIdx.x; v < m.V; v += blockDim.x) {
        float px, py;
        if (project32(c, vh + 3 * v, px, py)) {
            mnx = fminf(mnx, px); mny = fminf(mny, py);
            mxx = fmaxf(mxx, px); mxy = fmaxf(mxy, py);
        } else {
            bad = 1;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mnx = fminf(mnx, __shfl_xor(mnx, o)); mny = fminf(mny, __shfl_xor(mny, o));
        mxx = fmaxf(mxx, __shfl_xor(mxx, o)); mxy = fmaxf(mxy, __shfl_xor(mxy, o));
    }
    const int anybad = __syncthreads_or(bad);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { red[4 * w] = mnx; red[4 * w + 1] = mny; red[4 * w + 2] = mxx; red[4 * w + 3] = mxy; }
    __syncthreads();
    int tx0 = 0, ty0 = 0, nx = 0, ny = 0;
    {
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            mnx = fminf(mnx, red[4 * k]); mny = fminf(mny, red[4 * k + 1]);
            mxx = fmaxf(mxx, red[4 * k + 2]); mxy = fmaxf(mxy, red[4 * k + 3]);
        }
        const int ntx = (c.W + (1 << ts.tw_log2) - 1) >> ts.tw_log2;
        const int nty = (c.H + (1 << ts.th_log2) - 1) >> ts.th_log2;
        if (anybad) {
            nx = ntx; ny = nty;
        } else if (!(mxx < -1.0f || mxy < -1.0f || mnx > c.W + 1.0f || mny > c.H + 1.0f)) {
            // one pixel of margin around the float32 projections
            int x0 = (int)floorf(fmaxf(mnx - 1.0f, 0.0f)), y0 = (int)floorf(fmaxf(mny - 1.0f, 0.0f));
            int x1 = (int)floorf(fminf(mxx + 1.0f, (float)c.W - 1.0f));
            int y1 = (int)floorf(fminf(mxy + 1.0f, (float)c.H - 1.0f));
            tx0 = x0 >> ts.tw_log2; ty0 = y0 >> ts.th_log2;
            nx = (x1 >> ts.tw_log2) + 1 - tx0; ny = (y1 >> ts.th_log2) + 1 - ty0;
        }
    }
    const int count = (nx > 0 && ny > 0) ? nx * ny : 0;
    if (threadIdx.x == 0) {
        base = count > 0 ? atomicAdd(tile_count, count) : 0;
        // pixel rectangle covered by the view's tiles (empty if none)
        view_rect[vi] = count > 0 ? make_int4(tx0 << ts.tw_log2, ty0 << ts.th_log2,
                                                       min(c.W, (tx0 + nx) << ts.tw_log2),
                                                       min(c.H, (ty0 + ny) << ts.th_log2))
                                          : make_int4(0, 0, 0, 0);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < count; i += blockDim.x)
        tiles[base + i] = make_int2(vi, (tx0 + i % nx) | ((ty0 + i / nx) << 16));
}

// Inclusive prefix sum over the block (blockDim a multiple of 64, at most
// 1024); `wtot` is LDS [16].  Every thread of the block must call it.
__device__ __forceinline__ unsigned long long block_scan_u64(unsigned long long x, unsigned long long* wtot)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wtot[w] = x;
    __syncthreads();
    unsigned long long off = 0;
    for (int k = 0; k < w; ++k) off += wtot[k];
    __syncthreads();
    return x + off;
}

// Screen bins of view vi (one block, LDS `dyn`: the projected vertices, two
// counters per cell).  Every leaf slot's triangle gets padded screen bounds;
// triangles whose bounds touch the image are listed in every bin they touch.
// A bin's list runs from near to far in depth bands (the triangle's nearest
// vertex, bands spanning the hand's depth range in this view; inside a band
// the order is arbitrary), so a ray usually meets its hit early and skips the
// triangles behind it.  Lists are counted per (bin, band) cell, scanned, then
// filled by LDS cursors.  A view with a vertex less than 1 mm in front of the
// camera, more than kMaxBinsLds bins or more entries than the capacity is
// marked unbinned: its camera rays traverse the hierarchy.
__device__ void bin_view(const PrepArgs& a, int vi, float* dyn)
{
    __shared__ int bad;
    __shared__ float zred[2 * 16];
    __shared__ unsigned long long wtot[16];
    const ViewDev c = load_view(a.views, vi);
    const int V = a.m.V, F = a.m.F;
    const int lb = a.bins.log2;
    const int nbx = c.nbx, nby = (c.H + (1 << lb) - 1) >> lb, nb = nbx * nby;
    if (nb > kMaxBinsLds || !a.with_bins) {   // uniform over the block
        if (threadIdx.x == 0) a.bins.binned[vi] = 0;
        return;
    }
    int nband = kMaxBands;
    while (nband > 1 && nb * nband > kMaxBinCells) nband >>= 1;
    const int ncell = nb * nband;
    float* pxy = dyn;                                   // [V][3] px, py (screen), camera depth
    int* cnt = reinterpret_cast<int*>(pxy + 3 * V);     // [ncell] bin-major, band-minor
    int* cur = cnt + ncell;                             // [ncell]
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) cnt[k] = 0;
    const float* vg = a.verts + (size_t)c.hand * V * 3;
    int my_bad = 0;
    float zlo = 3e38f, zhi = -3e38f;
    for (int v = threadIdx.x; v < V; v += blockDim.x) {
        const float q0 = vg[3 * v] - c.o[0], q1 = vg[3 * v + 1] - c.o[1], q2 = vg[3 * v + 2] - c.o[2];
        const float xc = (c.R[0] * q0 + c.R[1] * q1) + c.R[2] * q2;
        const float yc = (c.R[3] * q0 + c.R[4] * q1) + c.R[5] * q2;
        const float zc = (c.R[6] * q0 + c.R[7] * q1) + c.R[8] * q2;
        if (!(zc > 1e-3f)) my_bad = 1;
        pxy[3 * v] = (c.fx * xc) / zc + c.cx;
        pxy[3 * v + 1] = (c.fy * yc) / zc + c.cy;
        pxy[3 * v + 2] = zc;
        zlo = fminf(zlo, zc);
        zhi = fmaxf(zhi, zc);
    }
    for (int o = 32; o > 0; o >>= 1) {
        zlo = fminf(zlo, __shfl_xor(zlo, o));
        zhi = fmaxf(zhi, __shfl_xor(zhi, o));
    }
    if ((threadIdx.x & 63) == 0) { zred[2 * (threadIdx.x >> 6)] = zlo; zred[2 * (threadIdx.x >> 6) + 1] = zhi; }
    if (__syncthreads_or(my_bad)) {
        if (threadIdx.x == 0) a.bins.binned[vi] = 0;
        return;
    }
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { zlo = fminf(zlo, zred[2 * k]); zhi = fmaxf(zhi, zred[2 * k + 1]); }
    const float zscale = (float)nband / fmaxf(zhi - zlo, 1e-6f);
    // padded bounds: far beyond the float32 rounding of the projections and
    // of the ray test (below 1e-3 px), and beyond the largest rounding of a
    // sample point onto a pixel's far edge
    const float pad = 1.0f / 16.0f;
    const int* sv = a.b.slot_verts + (size_t)c.hand * F * 3;
    float4* box = a.bins.box + (size_t)vi * F;
    auto bounds = [&](int i, float4& bx, int& x0, int& y0, int& x1, int& y1, int& band) -> bool {
        const float* p0 = pxy + 3 * sv[3 * i];
        const float* p1 = pxy + 3 * sv[3 * i + 1];
        const float* p2 = pxy + 3 * sv[3 * i + 2];
        bx.x = fminf(fminf(p0[0], p1[0]), p2[0]) - pad;
        bx.y = fminf(fminf(p0[1], p1[1]), p2[1]) - pad;
        bx.z = fmaxf(fmaxf(p0[0], p1[0]), p2[0]) + pad;
        bx.w = fmaxf(fmaxf(p0[1], p1[1]), p2[1]) + pad;
        band = min(nband - 1, max(0, (int)((fminf(fminf(p0[2], p1[2]), p2[2]) - zlo) * zscale)));
        if (bx.z < 0.0f || bx.w < 0.0f || bx.x > (float)c.W || bx.y > (float)c.H) return false;
        x0 = max(0, (int)floorf(bx.x)) >> lb;
        y0 = max(0, (int)floorf(bx.y)) >> lb;
        x1 = min(c.W - 1, (int)floorf(bx.z)) >> lb;
        y1 = min(c.H - 1, (int)floorf(bx.w)) >> lb;
        return true;
    };
    for (int i = threadIdx.x; i < F; i += blockDim.x) {
        float4 bx;
        int x0, y0, x1, y1, band;
        const bool in = bounds(i, bx, x0, y0, x1, y1, band);
        box[i] = bx;
        if (!in) continue;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) atomicAdd(cnt + (y * nbx + x) * nband + band, 1);
    }
    __syncthreads();
    // exclusive offsets of the cells: contiguous runs per thread, block scan of the runs
    const int per = (ncell + blockDim.x - 1) / blockDim.x;
    const int k0 = min(ncell, (int)threadIdx.x * per), k1 = min(ncell, k0 + per);
    unsigned long long local = 0;
    for (int k = k0; k < k1; ++k) local += (unsigned long long)cnt[k];
    const unsigned long long incl = block_scan_u64(local, wtot);
    unsigned long long run = incl - local;
    for (int k = k0; k < k1; ++k) {
        cur[k] = (int)run;
        run += (unsigned long long)cnt[k];
    }
    if (threadIdx.x == blockDim.x - 1) bad = incl > (unsigned long long)a.bins.cap;
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) a.bins.binned[vi] = 0;
        return;
    }
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const int first = cur[b * nband];
        const int last = cur[(b + 1) * nband - 1] + cnt[(b + 1) * nband - 1];
        a.bins.off[c.bin0 + b] = first;
        a.bins.count[c.bin0 + b] = last - first;
    }
    __syncthreads();   // the offsets are read before the cursors move
    uint16_t* ent = a.bins.entries + (size_t)vi * a.bins.cap;
    for (int i = threadIdx.x; i < F; i += blockDim.x) {
        float4 bx;
        int x0, y0, x1, y1, band;
        if (!bounds(i, bx, x0, y0, x1, y1, band)) continue;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) ent[atomicAdd(cur + (y * nbx + x) * nband + band, 1)] = (uint16_t)i;
    }
    if (threadIdx.x == 0) a.bins.binned[vi] = 1;
}

// number of non-zero bytes of a 16-byte word: bit 7 of each byte of
// ((w & 0x7F..) + 0x7F..) | w is set exactly when that byte is non-zero
__device__ __forceinline__ int nonzero_bytes(uint4 q)
{
    const unsigned int w[4] = {q.x, q.y, q.z, q.w};
    int c = 0;
    for (int k = 0; k < 4; ++k)
        c += __popc((((w[k] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w[k]) & 0x80808080u);
    return c;
}

// Loss scale of view vi from its mask: 1 / (3 * masked pixels), 0 if none
// (the value the loss kernels derive from their exact per-chunk counts).
__device__ void mask_scale(const ViewDev* __restrict__ views, const uint8_t* __restrict__ mask,
                           float* __restrict__ view_scale, int vi)
{
    __shared__ int red[16];
    const ViewDev c = views[vi];
    const long long n = (long long)c.W * c.H;
    long long cnt = 0;
    if (!mask) {
        cnt = threadIdx.x == 0 ? n : 0;
    } else {
        const uint8_t* mv = mask + c.pix0;
        // bytes up to a 16-byte boundary, then 16 at a time, then the tail
        const long long head = min(n, (long long)((16 - ((uintptr_t)mv & 15)) & 15));
        const long long n16 = (n - head) >> 4;
        for (long long i = threadIdx.x; i < head; i += blockDim.x) cnt += mv[i] != 0;
        const uint4* m16 = reinterpret_cast<const uint4*>(mv + head);
        // four 16-byte loads in flight per thread
        const long long s = blockDim.x;
        long long i = threadIdx.x;
        for (; i + 3 * s < n16; i += 4 * s) {
            const uint4 q[4] = {m16[i], m16[i + s], m16[i + 2 * s], m16[i + 3 * s]};
            for (int k = 0; k < 4; ++k) cnt += nonzero_bytes(q[k]);
        }
        for (; i < n16; i += s) cnt += nonzero_bytes(m16[i]);
        for (long long i = head + 16 * n16 + threadIdx.x; i < n; i += blockDim.x) cnt += mv[i] != 0;
    }
    int ci = (int)cnt;
    for (int o = 32; o > 0; o >>= 1) ci += __shfl_xor(ci, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ci;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long tot = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tot += red[k];
        const float tc = (float)tot;
        view_scale[vi] = tc > 0.0f ? 1.0f / (3.0f * tc) : 0.0f;
    }
}



// ===========================================================================
// render
// ===========================================================================

// iteration index of the sample streams: from device memory when the launch
// belongs to a device-counted (graph-replayable) iteration
__device__ __forceinline__ uint64_t iteration(const int* iter_dev, uint32_t iter)
{
    return iter_dev ? (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(*iter_dev) : (uint64_t)iter;
}

__device__ __forceinline__ uint64_t pick(const U64x4& r, int j)
{
    return j == 0 ? r.x[0] : j == 1 ? r.x[1] : j == 2 ? r.x[2] : r.x[3];
}

// Lane layout of a wave tile: lane = (pixel in tile) * G + sample, G = 2^spp_log2
// lanes per pixel; tiles of tw x th pixels.  Returns the lane's pixel.
__device__ __forceinline__ void tile_pixel(const TileShape& ts, int2 e, int lane, int& px, int& py)
{
    const int pit = lane >> ts.spp_log2;
    const int tx = e.y & 0xffff, ty = e.y >> 16;
    px = (tx << ts.tw_log2) + (pit & ((1 << ts.tw_log2) - 1));
    py = (ty << ts.th_log2) + (pit >> ts.tw_log2);
}

// Render the listed wave tiles; this block is `bid` of `nb` blocks sharing them.
// L1 loss gradient of one rendered pixel (the arithmetic of k_loss_grad)
__device__ __forceinline__ void pixel_dimage(const RenderArgs& a, int view, long long pg, const float* img)
{
    const bool on = !a.mask || a.mask[pg] != 0;
    const float sc = a.view_scale[view];
    for (int ch = 0; ch < 3; ++ch) {
        const float d = img[ch] - a.target[3 * pg + ch];
        const float sg = (float)((d > 0.0f) - (d < 0.0f));
        a.dimage[3 * pg + ch] = on ? sg * sc : 0.0f;
    }
}

// Pixels outside the views' tile rectangles get the background (and its loss
// gradient); the accumulators of a following backward pass are cleared
// (grid-stride work of the render blocks, beside the latency-bound tracing).
__device__ void render_side_work(const RenderArgs& a, int bid, int nb)
{
    const long long stride = (long long)nb * blockDim.x;
    const long long i0 = (long long)bid * blockDim.x + threadIdx.x;
    if (a.view_rect) {
        for (int v = 0; v < a.n_views; ++v) {
            const ViewDev& c = a.views[v];
            const int4 rc = a.view_rect[v];
            const long long np = (long long)c.W * c.H;
            for (long long pl = i0; pl < np; pl += stride) {
                const int py = (int)(pl / c.W), px = (int)(pl - (long long)py * c.W);
                if (px >= rc.x && px < rc.z && py >= rc.y && py < rc.w) continue;
                const long long pg = c.pix0 + pl;
                const float bg[3] = {a.background[3 * pg], a.background[3 * pg + 1], a.background[3 * pg + 2]};
                a.image[3 * pg] = bg[0];
                a.image[3 * pg + 1] = bg[1];
                a.image[3 * pg + 2] = bg[2];
                if (a.dimage) pixel_dimage(a, v, pg, bg);
            }
        }
    }
    for (int k = 0; k < 3; ++k) {
        float* p = a.clear[k];
        const long long n = a.clear_n[k];
        if (!p) continue;
        for (long long i = i0; i < n; i += stride) p[i] = 0.0f;
    }
}

// Wave tiles gw, gw + nw, ... (wave-uniform gw).  RASTER: hard rasterisation
// (a separate instantiation, so the ray tracer's register allocation does not
// carry the rasteriser's float64 state).  SPLIT > 1 (few tiles, ray tracing
// only): the SPLIT waves of a block render the same tiles, gw and nw then
// counting blocks; each walks every SPLIT-th touching triangle of the tile's
// screen bin, the partial closest hits meet in LDS (`xch`: two halves of
// SPLIT x 64 (t, face, slot) records, alternating per round, so that one
// barrier per round suffices) and the block's first wave takes their
// minimum, shades and writes the tile while the others go on.
template <bool COUNT, bool RASTER, int SPLIT = 1>
__device__ void render_tiles(const RenderArgs& a, int gw, int nw, int* stack, float* xch = nullptr)
{
    const uint64_t iter = iteration(a.iter_dev, a.iter);
    int* wst = stack + kMaxStack * (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int G = 1 << a.ts.spp_log2;
    const int s_lane = lane & (G - 1);
    const int n_tiles = *a.tile_count;
    const float inv_spp = 1.0f / (float)a.spp;
    const int wv = SPLIT > 1 ? (int)(threadIdx.x >> 6) : 0;   // the wave's part of each bin
    int xr = 0;                                               // exchanges so far (the LDS half)
    TraceCount tc;
    unsigned long long n_rays = 0, n_hit = 0;
    for (int t = gw; t < n_tiles; t += nw) {
        const int2 et = a.tiles[t];   // t is wave-uniform
        const int2 e = make_int2(__builtin_amdgcn_readfirstlane(et.x), __builtin_amdgcn_readfirstlane(et.y));
        const ViewDev& c = a.views[e.x];
        int px, py;
        tile_pixel(a.ts, e, lane, px, py);
        const bool pix_ok = px < c.W && py < c.H;
        const long long pl = (long long)py * c.W + px;
        const long long pg = c.pix0 + pl;
        const Node* nodes = a.nodes + (size_t)c.hand * a.n_nodes;
        const Tri* tris = a.tris + (size_t)c.hand * a.n_faces;
        const float* normals = a.normals + (size_t)c.hand * a.n_verts * 3;
        const float* tex = a.albedo + (size_t)c.hand * a.tex_h * a.tex_w * 3;
        const uint64_t c2 = (uint64_t)c.sid | (kDomainCamera << 32);
        // the tile's screen bin (all wave-uniform): an empty bin means every
        // sample of the tile misses, without a ray
        const int tx0 = (e.y & 0xffff) << a.ts.tw_log2, ty0 = (e.y >> 16) << a.ts.th_log2;
        const bool binned = __builtin_amdgcn_readfirstlane(a.bins.binned[e.x]) != 0;
        int bcnt = 0;
        const uint16_t* bent = nullptr;
        if (binned) {
            const int bb = c.bin0 + (tx0 >> a.bins.log2) + (ty0 >> a.bins.log2) * c.nbx;
            bcnt = __builtin_amdgcn_readfirstlane(a.bins.count[bb]);
            bent = a.bins.entries + (size_t)e.x * a.bins.cap + __builtin_amdgcn_readfirstlane(a.bins.off[bb]);
        }
        const bool empty = binned && bcnt == 0;
        const float4* bbox = a.bins.box + (size_t)e.x * a.n_faces;
        const float rx0 = (float)tx0, ry0 = (float)ty0;
        const float rx1 = (float)(tx0 + (1 << a.ts.tw_log2)), ry1 = (float)(ty0 + (1 << a.ts.th_log2));
        float acc[3] = {0.0f, 0.0f, 0.0f};
        int misses = 0;
        for (int r = 0; r < a.ts.rounds; ++r) {
            const int s = s_lane + 64 * r;
            const bool act = pix_ok && s < a.spp;
            float u = 0.0f, v = 0.0f;
            uint64_t wd = 0;
            if (act && !empty) {
                if (RASTER) {
                    wd = kCentreWord;
                } else {
                    const U64x4 rr = philox4x64((uint64_t)pl, (uint64_t)(s >> 2), c2, iter, a.seed, 0);
                    wd = pick(rr, s & 3);
                }
                u = u24_lo(wd);
                v = u24_hi(wd);
            }
            Hit h;
            h.face = -1;
            h.slot = 0;
            if (RASTER && !empty) {
                raster_list<COUNT>(tris, binned ? bent : nullptr, binned ? bcnt : a.n_faces, binned ? bbox : nullptr,
                                   rx0, ry0, rx1, ry1, c, (double)px + 0.5, (double)py + 0.5, act, h, &tc);
            } else if (!RASTER && !empty) {
                Ray ray;
                ray_screen(c, (float)px + u, (float)py + v, ray);
                if (binned)
                    trace_bins<COUNT, SPLIT>(tris, bent, bcnt, bbox, rx0, ry0, rx1, ry1, ray, act, h, &tc, wv);
                else if (wv == 0)
                    trace_wave<COUNT, true>(nodes, tris, ray, act, wst, h, &tc);
            }
            if (SPLIT > 1 && !empty) {
                // the block's partial hits (the tile, hence `empty`, is the
                // block's): lexicographic minimum of (t, face)
                float* x = xch + (size_t)(xr & 1) * SPLIT * 64 * 3;
                ++xr;
                float bt = h.face >= 0 ? h.t : __builtin_inff();
                int bf = h.face >= 0 ? h.face : 0x7fffffff, bs = h.slot;
                float* mine = x + (wv * 64 + lane) * 3;
                mine[0] = bt;
                mine[1] = __int_as_float(bf);
                mine[2] = __int_as_float(bs);
                __syncthreads();
                if (wv == 0) {
                    for (int k = 1; k < SPLIT; ++k) {
                        const float* o = x + (k * 64 + lane) * 3;
                        const float ot = o[0];
                        const int of = __float_as_int(o[1]);
                        if (ot < bt || (ot == bt && of < bf)) {
                            bt = ot;
                            bf = of;
                            bs = __float_as_int(o[2]);
                        }
                    }
                    h.face = bf == 0x7fffffff ? -1 : bf;
                    h.slot = bs;
                    h.t = bt;
                }
            }
            if (SPLIT > 1 && wv != 0) continue;   // shading and writes: the block's first wave
            if (act) {
                if (COUNT && !empty) ++n_rays;
                if (a.hit_face) a.hit_face[pg * a.spp + s] = h.face;
                if (a.hit_rec) a.hit_rec[((size_t)t * a.ts.rounds + r) * 64 + lane] = hit_record(wd, h.face >= 0 ? h.slot : -1);
                if (h.face >= 0) {
                    if (COUNT) ++n_hit;
                    Surf sf;
                    surface(tris, a.uv, h.slot, c, px + (double)u, py + (double)v, sf);
                    Shade sd;
                    shade_hit(sf, normals, a.uv, tex, a.tex_h, a.tex_w, a.shading, sd);
                    for (int ch = 0; ch < 3; ++ch) acc[ch] += sd.col[ch] * sd.shade;
                } else {
                    ++misses;
                }
            }
        }
        if (SPLIT > 1 && wv != 0) continue;
        // sum over the G lanes of the pixel (fixed butterfly order)
        for (int o = G >> 1; o > 0; o >>= 1) {
            acc[0] += __shfl_xor(acc[0], o);
            acc[1] += __shfl_xor(acc[1], o);
            acc[2] += __shfl_xor(acc[2], o);
            misses += __shfl_xor(misses, o);
        }
        if (s_lane == 0 && pix_ok) {
            const float* bg = a.background + 3 * pg;
            float out[3];
            if (misses == a.spp) {
                out[0] = bg[0]; out[1] = bg[1]; out[2] = bg[2];
            } else {
                const float fm = (float)misses;
                for (int ch = 0; ch < 3; ++ch) out[ch] = (acc[ch] + fm * bg[ch]) * inv_spp;
            }
            a.image[3 * pg] = out[0];
            a.image[3 * pg + 1] = out[1];
            a.image[3 * pg + 2] = out[2];
            if (a.dimage) pixel_dimage(a, e.x, pg, out);
        }
    }
    if (COUNT) {
        atomicAdd(a.counts + 0, n_rays);
        atomicAdd(a.counts + 1, (unsigned long long)tc.nodes);
        atomicAdd(a.counts + 2, (unsigned long long)tc.tris);
        atomicAdd(a.counts + 3, n_hit);
        atomicAdd(a.counts + 4, (unsigned long long)tc.nodes_w);
        atomicAdd(a.counts + 5, (unsigned long long)tc.tris_w);
    }
}

// ===========================================================================
// L1 loss
// ===========================================================================

// partial sums of chunk ck: |image - target| over masked pixels and the
// masked-pixel count (blocks of 256 threads)
__device__ void loss_partial(const LossArgs& a, int chunk)
{
    __shared__ float red[2 * 16];
    const int2 ck = a.chunks[chunk];   // (view, first pixel in view)
    const ViewDev c = a.views[ck.x];
    const long long n = (long long)c.W * c.H;
    float s = 0.0f, cnt = 0.0f;
    for (int k = threadIdx.x; k < kLossChunk; k += blockDim.x) {
        long long pl = (long long)ck.y + k;
        if (pl >= n) break;
        long long pg = c.pix0 + pl;
        if (a.mask && a.mask[pg] == 0) continue;
        if (a.image)
            s += fabsf(a.image[3 * pg] - a.target[3 * pg]) + fabsf(a.image[3 * pg + 1] - a.target[3 * pg + 1]) +
                 fabsf(a.image[3 * pg + 2] - a.target[3 * pg + 2]);
        cnt += 1.0f;
    }
    s = wave_sum(s);
    cnt = wave_sum(cnt);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { red[2 * w] = s; red[2 * w + 1] = cnt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        float ts = 0.0f, tc = 0.0f;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { ts += red[2 * k]; tc += red[2 * k + 1]; }
        a.partial[2 * chunk] = ts;
        a.partial[2 * chunk + 1] = tc;
    }
}

__global__ void __launch_bounds__(256) k_loss_partial(LossArgs a)
{
    loss_partial(a, blockIdx.x);
}

// Hand h: per view, the chunk partials summed in a fixed order by the first
// 256 threads (the block may be larger; all of it reaches the barriers).
__device__ void loss_final(const LossArgs& a, int h)
{
    __shared__ float red[2 * 4];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    float loss = 0.0f;
    for (int q = a.hand_view_off[h]; q < a.hand_view_off[h + 1]; ++q) {
        const int v = a.hand_views[q];
        float s = 0.0f, cnt = 0.0f;
        if (t < 256)
            for (int k = a.view_chunk_off[v] + t; k < a.view_chunk_off[v + 1]; k += 256) {
                s += a.partial[2 * k];
                cnt += a.partial[2 * k + 1];
            }
        s = wave_sum(s);
        cnt = wave_sum(cnt);
        if (lane == 0 && w < 4) { red[2 * w] = s; red[2 * w + 1] = cnt; }
        __syncthreads();
        if (t == 0) {
            float ts = 0.0f, tc = 0.0f;
            for (int k = 0; k < 4; ++k) { ts += red[2 * k]; tc += red[2 * k + 1]; }
            if (a.view_scale) a.view_scale[v] = tc > 0.0f ? 1.0f / (3.0f * tc) : 0.0f;
            if (tc > 0.0f) loss += ts / (3.0f * tc);
        }
        __syncthreads();
    }
    if (t == 0 && a.loss) a.loss[h] = loss;
}

// one block (256 threads) per hand
__global__ void __launch_bounds__(256) k_loss_final(LossArgs a)
{
    loss_final(a, blockIdx.x);
}

// Loss value of hand h from the chunk partials inside a block of up to 16
// waves: one wave per view, the views then added in order.
__device__ void loss_value_hand(const LossArgs& a, int h)
{
    __shared__ float red[2 * 16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int nw = min((int)(blockDim.x >> 6), 16);
    const int q0 = a.hand_view_off[h], q1 = a.hand_view_off[h + 1];
    float loss = 0.0f;
    for (int qb = q0; qb < q1; qb += nw) {
        const int q = qb + w;
        float s = 0.0f, cnt = 0.0f;
        if (w < nw && q < q1) {
            const int v = a.hand_views[q];
            for (int k = a.view_chunk_off[v] + lane; k < a.view_chunk_off[v + 1]; k += 64) {
                s += a.partial[2 * k];
                cnt += a.partial[2 * k + 1];
            }
        }
        s = wave_sum(s);
        cnt = wave_sum(cnt);
        if (lane == 0 && w < nw) { red[2 * w] = s; red[2 * w + 1] = cnt; }
        __syncthreads();
        if (t == 0)
            for (int k = 0; k < nw && qb + k < q1; ++k)
                if (red[2 * k + 1] > 0.0f) loss += red[2 * k] / (3.0f * red[2 * k + 1]);
        __syncthreads();
    }
    if (t == 0) a.loss[h] = loss;
}

__global__ void __launch_bounds__(256) k_loss_grad(LossArgs a)
{
    const int2 ck = a.chunks[blockIdx.x];
    const ViewDev c = a.views[ck.x];
    const long long n = (long long)c.W * c.H;
    const float sc = a.view_scale[ck.x];
    for (int k = threadIdx.x; k < kLossChunk; k += blockDim.x) {
        long long pl = (long long)ck.y + k;
        if (pl >= n) break;
        long long pg = c.pix0 + pl;
        bool on = !a.mask || a.mask[pg] != 0;
        for (int ch = 0; ch < 3; ++ch) {
            float d = a.image[3 * pg + ch] - a.target[3 * pg + ch];
            float sg = (float)((d > 0.0f) - (d < 0.0f));
            a.dimage[3 * pg + ch] = on ? sg * sc : 0.0f;
        }
    }
}

// ===========================================================================
// interior adjoint
// ===========================================================================

constexpr int kStageW = 11;   // staged scatter of one sample's colour-map footprint: 4 texels, 4 weights, RGB

// Interior adjoint over the listed wave tiles; block `bid` of `nb`.
template <bool COUNT>
__device__ void adjoint_tiles(const AdjointArgs& a, int bid, int nb, int* stack, float* patch_base, float* stage)
{
    const uint64_t iter = iteration(a.iter_dev, a.iter);
    // this wave's four row windows, zero between uses (the flush clears what it reads)
    float* patch = patch_base + kWaveWin * (threadIdx.x >> 6);
    {
        float4* z = reinterpret_cast<float4*>(patch);
        for (int f = threadIdx.x & 63; f < kWaveWin / 4; f += 64) z[f] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        wave_lds_sync();
    }
    int* wst = stack + kMaxStack * (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int G = 1 << a.ts.spp_log2;
    const int s_lane = lane & (G - 1);
    const int gw = __builtin_amdgcn_readfirstlane((int)((bid * kThreads + threadIdx.x) >> 6));
    const int nw = (int)((nb * kThreads) >> 6);
    const int n_tiles = *a.tile_count;
    const float inv_spp = 1.0f / (float)a.spp;
    const Shading S = a.shading;
    // hits stored by the render of the same geometry and iteration: no re-trace
    const bool stored = a.hit_rec != nullptr && __builtin_amdgcn_readfirstlane(*a.hit_iter) == (int)iter;
    TraceCount tc;
    unsigned long long n_rays = 0, n_hit = 0;
    // wave-uniform tile entries through the scalar cache, the next one
    // fetched while the current tile is worked on
    const ConstI* tl = (const ConstI*)a.tiles;
    int2 e_nx = make_int2(0, 0);
    if (gw < n_tiles) e_nx = make_int2(tl[2 * gw], tl[2 * gw + 1]);
    for (int t = gw; t < n_tiles; t += nw) {
        const int2 e = e_nx;
        if (t + nw < n_tiles) e_nx = make_int2(tl[2 * (t + nw)], tl[2 * (t + nw) + 1]);
        const ViewDev& c = a.views[e.x];
        int px, py;
        tile_pixel(a.ts, e, lane, px, py);
        const bool pix_ok = px < c.W && py < c.H;
        const long long pl = (long long)py * c.W + px;
        const long long pg = c.pix0 + pl;
        float g[3] = {0.0f, 0.0f, 0.0f};
        if (pix_ok) {
            g[0] = a.dimage[3 * pg] * inv_spp;
            g[1] = a.dimage[3 * pg + 1] * inv_spp;
            g[2] = a.dimage[3 * pg + 2] * inv_spp;
        }
        const bool live = g[0] != 0.0f || g[1] != 0.0f || g[2] != 0.0f;
        if (!__any(live)) continue;   // wave-uniform
        const int hand = c.hand;
        const Node* nodes = a.nodes + (size_t)hand * a.n_nodes;
        const Tri* tris = a.tris + (size_t)hand * a.n_faces;
        const float* normals = a.normals + (size_t)hand * a.n_verts * 3;
        const float* tex = a.albedo + (size_t)hand * a.tex_h * a.tex_w * 3;
        float* gtex = a.grad_albedo + (size_t)hand * a.tex_h * a.tex_w * 3;
        const uint64_t c2 = (uint64_t)c.sid | (kDomainCamera << 32);
        for (int r = 0; r < a.ts.rounds; ++r) {
            const int s = s_lane + 64 * r;
            // per-sample contributions to the triangle's three vertices:
            // [k*3 + c] position gradient, [9 + k*3 + c] normal gradient
            float gv[18];
            for (int k = 0; k < 18; ++k) gv[k] = 0.0f;
            int face = -1;
            int tidx[4] = {0, 0, 0, 0};   // texels of the bilinear footprint
            float twt[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            int tmask = 0;
            int fi0 = 0x7fffffff, fi1 = -1, fj0 = 0x7fffffff, fj1 = -1;   // footprint rows / columns
            const bool act = live && s < a.spp;
            // a stored hit record carries the sample's random word: no
            // Philox here; re-traced samples draw it again
            const uint64_t rec = stored && act ? a.hit_rec[((size_t)t * a.ts.rounds + r) * 64 + lane] : 0ull;
            const int slot = stored && act ? hit_record_slot(rec) : -1;
            if (stored && !__any(slot >= 0)) continue;   // no hit in this round of the tile
            uint64_t wd = rec;
            if (!stored) {
                const U64x4 rr = philox4x64((uint64_t)pl, (uint64_t)(s >> 2), c2, iter, a.seed, 0);
                wd = pick(rr, s & 3);
            }
            const float u = act ? u24_lo(wd) : 0.0f, v = act ? u24_hi(wd) : 0.0f;
            Hit h;
            if (stored) {
                h.slot = slot;
                h.face = slot;   // >= 0 for a hit; the face id comes with the triangle below
            } else {
                Ray ray;
                ray_screen(c, (float)px + u, (float)py + v, ray);
                trace_wave<COUNT, true>(nodes, tris, ray, act, wst, h, &tc);
            }
            if (act) {
                if (COUNT && !stored) ++n_rays;   // rays traced again (stored hits are read, not traced)
                if (h.face >= 0) {
                    if (COUNT) ++n_hit;
                    Surf sf;
                    surface(tris, a.uv, h.slot, c, px + (double)u, py + (double)v, sf);
                    face = sf.face;
                    Shade sd;
                    shade_hit(sf, normals, a.uv, tex, a.tex_h, a.tex_w, S, sd);
                    for (int k = 0; k < 4; ++k) {
                        tidx[k] = sd.idx[k];
                        twt[k] = sd.shade * sd.w[k];
                    }
                    tmask = 0xF;
                    fi0 = sd.ti0; fi1 = sd.ti1; fj0 = sd.tj0; fj1 = sd.tj1;
                    const float gs = g[0] * sd.col[0] + g[1] * sd.col[1] + g[2] * sd.col[2];
                    float gtu = 0.0f, gtv = 0.0f;
                    for (int ch = 0; ch < 3; ++ch) {
                        gtu += g[ch] * sd.shade * sd.dcol_du[ch];
                        gtv += g[ch] * sd.shade * sd.dcol_dv[ch];
                    }
                    const float2 uv0 = *reinterpret_cast<const float2*>(a.uv + 2 * sf.i0);
                    const float2 uv1 = *reinterpret_cast<const float2*>(a.uv + 2 * sf.i1);
                    const float2 uv2 = *reinterpret_cast<const float2*>(a.uv + 2 * sf.i2);
                    float gb1 = gtu * (uv1.x - uv0.x) + gtv * (uv1.y - uv0.y);
                    float gb2 = gtu * (uv2.x - uv0.x) + gtv * (uv2.y - uv0.y);
                    if (sd.ndotl > 0.0f) {
                        float gn[3] = {gs * S.kd * S.l[0], gs * S.kd * S.l[1], gs * S.kd * S.l[2]};
                        const float gnn = gn[0] * sd.n[0] + gn[1] * sd.n[1] + gn[2] * sd.n[2];
                        const float inl = 1.0f / sd.nlen;
                        const float* n0 = normals + 3 * sf.i0;
                        const float* n1 = normals + 3 * sf.i1;
                        const float* n2 = normals + 3 * sf.i2;
                        for (int k = 0; k < 3; ++k) {
                            const float gr = (gn[k] - gnn * sd.n[k]) * inl;
                            gv[9 + k] = sf.b0 * gr;
                            gv[12 + k] = sf.b1 * gr;
                            gv[15 + k] = sf.b2 * gr;
                            gb1 += gr * (n1[k] - n0[k]);
                            gb2 += gr * (n2[k] - n0[k]);
                        }
                    }
                    // hit point: y = M^{-T} [gb1, gb2, 0], M = [v1-v0, v2-v0, -d] (float64);
                    // M's cofactor column (v2-v0) x (-d) = d x (v2-v0) and 1/det M
                    // come with the surface point's solve
                    double e1[3], md[3];
                    for (int k = 0; k < 3; ++k) {
                        e1[k] = (double)sf.v[3 + k] - (double)sf.v[k];
                        md[k] = -sf.d[k];
                    }
                    const double* c23 = sf.pv;
                    const double c31[3] = {md[1] * e1[2] - md[2] * e1[1], md[2] * e1[0] - md[0] * e1[2],
                                           md[0] * e1[1] - md[1] * e1[0]};
                    const double idet = sf.idet;
                    for (int k = 0; k < 3; ++k) {
                        const float y = (float)(((double)gb1 * c23[k] + (double)gb2 * c31[k]) * idet);
                        gv[k] = -sf.b0 * y;
                        gv[3 + k] = -sf.b1 * y;
                        gv[6 + k] = -sf.b2 * y;
                    }
                }
            }
            // Triangles: sum the lanes' contributions per triangle (a wave's
            // samples hit a few) and let one lane scatter each sum into the
            // triangle's slot [corner k][dL/dv (3), dL/dn (3)].  The sums run
            // on the DPP network and end in lane 63; lane `entry` takes
            // entry `entry` of the slot, so one instruction writes all 18.
            unsigned long long pending = __ballot(face >= 0);
            while (pending) {
                const int leader = __ffsll((long long)pending) - 1;
                const int f = __builtin_amdgcn_readlane(face, leader);
                const bool mine = face == f;
                pending &= ~__ballot(mine);
                float sv[18];
#pragma unroll
                for (int k = 0; k < 18; ++k) sv[k] = mine ? gv[k] : 0.0f;
                wave_sum63_n<18>(sv);   // the 18 sums interleaved
                float mine_val = 0.0f;
#pragma unroll
                for (int k = 0; k < 18; ++k) {
                    const float x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sv[k]), 63));
                    const int corner = k < 9 ? k / 3 : (k - 9) / 3;
                    const int entry = 6 * corner + (k < 9 ? k % 3 : 3 + (k - 9) % 3);
                    if (lane == entry) mine_val = x;
                }
                if (lane < 18) unsafeAtomicAdd(a.gface + ((size_t)hand * a.n_faces + f) * 18 + lane, mine_val);
            }
            // Colour map: each row of 16 lanes sums its samples' bilinear
            // footprints into an LDS window of up to W x W texels, then
            // adds the window's used part to the gradient, consecutive lanes
            // on consecutive floats, clearing it for the next use.  Where the
            // row's lanes all belong to one pixel (G >= 16) they share dL/dI
            // and the window holds one weight per texel (dL/dI is applied in
            // the flush, W = kWin); otherwise it holds RGB (W = kWinRGB).  Rows whose footprint does
            // not fit (a texture seam inside the row) scatter directly.
            const bool scalar = G >= 16;
            const int wr0 = row_min(fi0), wr1 = row_max(fi1);
            const int wc0 = row_min(fj0), wc1 = row_max(fj1);
            const int W = scalar ? kWin : kWinRGB;
            const bool fits = wr1 >= wr0 && wr1 - wr0 < W && wc1 - wc0 < W;   // uniform in the row
            float* win = patch + (lane >> 4) * (kWin * kWin);
            if (tmask && fits) {
                // start at corner (lane & 3): lanes sharing a footprint hit
                // different LDS words in each of the four steps
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int k = (q + lane) & 3;
                    const int ri = (k & 2) ? fi1 : fi0, rj = (k & 1) ? fj1 : fj0;
                    const float wk = k == 0 ? twt[0] : k == 1 ? twt[1] : k == 2 ? twt[2] : twt[3];
                    const int cell = (ri - wr0) * W + (rj - wc0);
                    if (scalar) {
                        atomicAdd(win + cell, wk);
                    } else {
                        atomicAdd(win + 3 * cell + 0, g[0] * wk);
                        atomicAdd(win + 3 * cell + 1, g[1] * wk);
                        atomicAdd(win + 3 * cell + 2, g[2] * wk);
                    }
                }
                tmask = 0;
            }
            wave_lds_sync();
            // flush: each row's 16 lanes walk its window's used part (the
            // row's lanes hold the same bounds and, with G >= 16, the same
            // dL/dI); row y, float x3 of the window from f via a float
            // reciprocal, exact here (f < 3 kWin^2, distance to the next
            // integer at least 1/(2 ncol))
            if (fits) {
                const int ncol = 3 * (wc1 - wc0 + 1), n = (wr1 - wr0 + 1) * ncol;
                const float rn = 1.0f / (float)ncol;
                float* wrow = patch + (lane >> 4) * (kWin * kWin);
                float* grow = gtex + 3 * ((size_t)wr0 * a.tex_w + wc0);
                for (int f = lane & 15; f < n; f += 16) {
                    const int y = (int)(((float)f + 0.5f) * rn);
                    const int x3 = f - ncol * y;
                    float x;
                    if (scalar) {
                        const int xt = x3 / 3, ch = x3 - 3 * xt;
                        float* cell = wrow + y * kWin + xt;
                        const float w = *cell;
                        // the texel's last channel clears it (its other two
                        // channels are read by lower f, no later)
                        if (ch == 2) *cell = 0.0f;
                        x = w * (ch == 0 ? g[0] : ch == 1 ? g[1] : g[2]);
                    } else {
                        float* cell = wrow + y * (3 * kWinRGB) + x3;
                        x = *cell;
                        *cell = 0.0f;
                    }
                    if (x != 0.0f) unsafeAtomicAdd(grow + (size_t)y * 3 * a.tex_w + x3, x);
                }
            }
            wave_lds_sync();
            // Footprints that did not fit their row's window (minified maps:
            // a few spp per pixel spread over many texels): a sample's twelve
            // values are two texel rows of two texels x RGB, six consecutive
            // floats when the columns are adjacent.  Staged in LDS, they are
            // scattered six lanes to a texel row, so that each atomic
            // instruction's lanes fall on a few cache lines (a lane per
            // sample puts each of twelve instructions on up to 64 lines).
            const uint64_t smask = __ballot(tmask != 0);
            if (smask) {
                float* st = stage + (threadIdx.x >> 6) * (64 * kStageW);
                if (tmask) {
                    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(smask >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)smask, 0u));
                    float* e = st + rank * kStageW;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        e[k] = __int_as_float(tidx[k]);
                        e[4 + k] = twt[k];
                    }
                    e[8] = g[0];
                    e[9] = g[1];
                    e[10] = g[2];
                }
                wave_lds_sync();
                const int njobs = 2 * __popcll(smask);   // (sample, texel row)
                const int jq = lane / 6, el = lane - 6 * jq;
                const int k_el = el >= 3 ? 1 : 0, ch = el - 3 * k_el;
                for (int q0 = 0; q0 < njobs; q0 += 10) {
                    const int q = q0 + jq;
                    if (jq < 10 && q < njobs) {
                        const float* e = st + (q >> 1) * kStageW;
                        const int k = 2 * (q & 1) + k_el;
                        const float x = e[8 + ch] * e[4 + k];
                        if (x != 0.0f) unsafeAtomicAdd(gtex + 3 * (size_t)__float_as_int(e[k]) + ch, x);
                    }
                }
                wave_lds_sync();   // the stage is written again by the next round
            }
        }
    }
    if (COUNT) {
        atomicAdd(a.counts + 0, n_rays);
        atomicAdd(a.counts + 1, (unsigned long long)tc.nodes);
        atomicAdd(a.counts + 2, (unsigned long long)tc.tris);
        atomicAdd(a.counts + 3, n_hit);
        atomicAdd(a.counts + 4, (unsigned long long)tc.nodes_w);
        atomicAdd(a.counts + 5, (unsigned long long)tc.tris_w);
    }
}

// ===========================================================================
// silhouette edges: classification, quantised weights, prefix sums
// ===========================================================================

// Exclusive prefix of the views' edge-sample budgets, prefix[n_views] the
// total (one block; budgets read past the L1, since other blocks of the same
// launch may have written them).
__device__ void budget_prefix(const long long* budget, int n_views, long long* prefix, unsigned long long* wtot)
{
    const int per = (n_views + blockDim.x - 1) / blockDim.x;
    const int v0 = min(n_views, (int)threadIdx.x * per), v1 = min(n_views, v0 + per);
    long long s = 0;
    for (int v = v0; v < v1; ++v) s += __hip_atomic_load(budget + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long incl = (long long)block_scan_u64((unsigned long long)s, wtot);
    long long run = incl - s;
    for (int v = v0; v < v1; ++v) {
        prefix[v] = run;
        run += __hip_atomic_load(budget + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x == blockDim.x - 1) prefix[n_views] = incl;
}

// exclusive prefix of the per-view edge-sample budgets (one block)
__global__ void __launch_bounds__(256) k_edge_prefix(const long long* __restrict__ budget, int n_views,
                                                     long long* __restrict__ prefix)
{
    __shared__ unsigned long long wtot[16];
    budget_prefix(budget, n_views, prefix, wtot);
}

// Silhouette table of view `vi` (one block; LDS from `part`: [16] scan
// buffer, the hand's vertices, each edge's weight).  The block that finishes
// last also writes the budget prefix over the views (`done` counts finished
// views and is left at zero).
__device__ void edges_setup_view(const EdgeArgs& a, int vi, unsigned long long* part, int* done)
{
    const ViewDev c = a.views[vi];
    const float* vg = a.verts + (size_t)c.hand * a.m.V * 3;
    const int E = a.m.E, V = a.m.V;
    EdgeRec* rec = a.rec + (size_t)vi * E;
    unsigned long long* cdf = a.cdf + (size_t)vi * E;
    float* vh = reinterpret_cast<float*>(part + 16);
    uint32_t* wl = reinterpret_cast<uint32_t*>(vh + 3 * V);
    __shared__ int last;
    lds_stage(vh, vg, 3 * V);
    __syncthreads();
    // weights, one edge per thread and pass (the next pass's table entry
    // fetched ahead)
    int4 n0 = make_int4(0, 0, 0, 0), n1 = n0;
    if ((int)threadIdx.x < E) { n0 = a.m.edge_verts[2 * threadIdx.x]; n1 = a.m.edge_verts[2 * threadIdx.x + 1]; }
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
        const int4 t0 = n0, t1 = n1;
        const int en = e + blockDim.x;
        if (en < E) { n0 = a.m.edge_verts[2 * en]; n1 = a.m.edge_verts[2 * en + 1]; }
        EdgeRec r;
        r.ax = r.ay = r.bx = r.by = r.t0 = r.t1 = 0.0f;
        r.w = 0; r.wq = 0;
        const int va = t0.x, vb = t0.y;
        const int fv[2][3] = {{t0.z, t0.w, t1.x}, {t1.y, t1.z, t1.w}};
        const float* pa = vh + 3 * va;
        int front[2] = {0, 0};
        const int nf = fv[1][0] < 0 ? 1 : 2;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (k >= nf) break;
            const float* p0 = vh + 3 * fv[k][0];
            const float* p1 = vh + 3 * fv[k][1];
            const float* p2 = vh + 3 * fv[k][2];
            float u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
            float w[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
            float n0x = u[1] * w[2] - u[2] * w[1];
            float n1x = u[2] * w[0] - u[0] * w[2];
            float n2x = u[0] * w[1] - u[1] * w[0];
            float w0 = c.o[0] - pa[0], w1 = c.o[1] - pa[1], w2 = c.o[2] - pa[2];
            float dd = (n0x * w0 + n1x * w1) + n2x * w2;
            front[k] = dd > 0.0f;
        }
        const bool sil = nf == 1 || front[0] != front[1];
        float ax, ay, bx, by;
        if (sil && project32(c, pa, ax, ay) && project32(c, vh + 3 * vb, bx, by)) {
            // Liang-Barsky clip to [0,W] x [0,H]
            float dx = bx - ax, dy = by - ay;
            float lo = 0.0f, hi = 1.0f;
            const float pp[4] = {-dx, dx, -dy, dy};
            const float qq[4] = {ax, (float)c.W - ax, ay, (float)c.H - ay};
            bool ok = true;
            for (int k = 0; k < 4; ++k) {
                if (pp[k] == 0.0f) {
                    if (qq[k] < 0.0f) ok = false;
                } else {
                    float rr = qq[k] / pp[k];
                    if (pp[k] < 0.0f) { if (rr > lo) lo = rr; }
                    else { if (rr < hi) hi = rr; }
                }
            }
            const float len = sqrtf(dx * dx + dy * dy);
            if (ok && lo < hi && len > 0.0f) {
                float ell = len * (hi - lo);
                float qv = floorf(ell * 256.0f);
                uint32_t wq = qv >= 4294967295.0f ? 0xFFFFFFFFu : (uint32_t)qv;
                if (wq == 0) wq = 1;
                r.ax = ax; r.ay = ay; r.bx = bx; r.by = by; r.t0 = lo; r.t1 = hi; r.w = wq; r.wq = wq;
            }
        }
        rec[e] = r;
        wl[e] = r.w;
    }
    __syncthreads();
    // integer CDF: contiguous runs of edges per thread, block scan of the
    // runs' sums
    const int per = (E + blockDim.x - 1) / blockDim.x;
    const int e0 = min(E, (int)threadIdx.x * per);
    const int e1 = min(E, e0 + per);
    unsigned long long local = 0;
    for (int e = e0; e < e1; ++e) local += wl[e];
    const unsigned long long incl = block_scan_u64(local, part);
    unsigned long long run = incl - local;
    for (int e = e0; e < e1; ++e) {
        run += wl[e];
        cdf[e] = run;
    }
    if (threadIdx.x == blockDim.x - 1) {
        a.total[vi] = incl;
        const unsigned long long div = (unsigned long long)a.budget_div;
        a.budget[vi] = (long long)((incl + div - 1ull) / div);
        __threadfence();
        last = atomicAdd(done, 1) == a.n_views - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    budget_prefix(a.budget, a.n_views, a.prefix, part);
    if (threadIdx.x == 0) *done = 0;
}

// Geometry preparation in one launch: blocks [0, H) refit hand h (triangles
// in leaf order, hierarchy bounds), blocks [H, 2H) its vertex normals; then per view the
// silhouette table (with_setup; the last one also the budget prefix), the screen bounds and wave tiles (the tile
// count is zero beforehand), the screen bins and the loss scale from the mask (with_scale).
__global__ void __launch_bounds__(512) k_prepare(PrepArgs a)
{
    extern __shared__ float dyn[];
    int bid = blockIdx.x;
    if (bid < a.n_hands) {
        refit_hand(a.m, a.b, a.verts, a.tris, a.nodes, bid, dyn, a.bvh_cost);
        return;
    }
    bid -= a.n_hands;
    if (bid < a.n_hands) {
        normals_hand(a.m, a.verts, a.normals, bid, dyn);
        return;
    }
    bid -= a.n_hands;
    if (a.with_setup) {
        if (bid < a.n_views) {
            edges_setup_view(a.e, bid, reinterpret_cast<unsigned long long*>(dyn), a.setup_done);
            return;
        }
        bid -= a.n_views;
    }
    if (bid < a.n_views) {
        view_bounds(a.m, a.views, a.verts, a.ts, a.tiles, a.tile_count, a.view_rect, bid);
        return;
    }
    bid -= a.n_views;
    if (bid < a.n_views) {
        bin_view(a, bid, dyn);
        return;
    }
    bid -= a.n_views;
    if (a.with_scale && bid < a.n_views) mask_scale(a.views, a.mask, a.view_scale, bid);
}

// ===========================================================================
// edge sampling (boundary term)
// ===========================================================================

__device__ __forceinline__ void shade_or_bg(const Hit& h, const Tri* tris, const ViewDev& c, float X, float Y,
                                            const float* normals, const float* uv, const float* tex, int th,
                                            int tw, const Shading& S, const float* bg, float* out)
{
    if (h.face >= 0) {
        Surf sf;
        surface(tris, uv, h.slot, c, (double)X, (double)Y, sf);
        Shade sd;
        shade_hit(sf, normals, uv, tex, th, tw, S, sd);
        for (int ch = 0; ch < 3; ++ch) out[ch] = sd.col[ch] * sd.shade;
    } else {
        for (int ch = 0; ch < 3; ++ch) out[ch] = bg[ch];
    }
}

// float64 projection of a vertex to the screen and its Jacobian d(px,py)/dv
__device__ __forceinline__ void project64(const ViewDev& c, const float* v, double p[2], double J[2][3])
{
    const double q[3] = {(double)v[0] - (double)c.o[0], (double)v[1] - (double)c.o[1], (double)v[2] - (double)c.o[2]};
    double xc[3];
    for (int r = 0; r < 3; ++r)
        xc[r] = (double)c.R[3 * r] * q[0] + (double)c.R[3 * r + 1] * q[1] + (double)c.R[3 * r + 2] * q[2];
    const double z = xc[2];
    p[0] = (double)c.fx * xc[0] / z + (double)c.cx;
    p[1] = (double)c.fy * xc[1] / z + (double)c.cy;
    const double d[2][3] = {{(double)c.fx / z, 0.0, -(double)c.fx * xc[0] / (z * z)},
                            {0.0, (double)c.fy / z, -(double)c.fy * xc[1] / (z * z)}};
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 3; ++k)
            J[r][k] = d[r][0] * (double)c.R[k] + d[r][1] * (double)c.R[3 + k] + d[r][2] * (double)c.R[6 + k];
}

// Geometry of edge sample kg (global index over the views' budgets): the
// view, the stratum of the view's integer CDF, the chosen edge and point, the
// unit screen normal, the side point of this lane (even lane x + delta n, odd
// lane x - delta n), the owning pixel and the weight factor (stratum width) /
// wq: the sample's weight is the edge's clipped length times it (stratum
// probability over point density).
struct EdgePoint {
    int vi, e;
    bool valid;          // false: empty stratum (no sample)
    float t, nhx, nhy, xs, ys, wgt;
    long long pg;
};

__device__ __forceinline__ void edge_point(const EdgeArgs& a, long long kg, uint64_t iter, int side, EdgePoint& P)
{
    const int E = a.m.E;
    // view of global sample kg: last v with prefix[v] <= kg
    int vlo = 0, vhi = a.n_views - 1;
    while (vlo < vhi) {
        const int mid = (vlo + vhi + 1) >> 1;
        if (a.prefix[mid] <= kg) vlo = mid; else vhi = mid - 1;
    }
    const int vi = vlo;
    P.vi = vi;
    const long long k = kg - a.prefix[vi];
    const long long M = a.budget[vi];
    const unsigned long long T = a.total[vi];
    const ViewDev& c = a.views[vi];
    const EdgeRec* rec = a.rec + (size_t)vi * E;
    const unsigned long long* cdf = a.cdf + (size_t)vi * E;
    const uint64_t c2 = (uint64_t)c.sid | (kDomainEdge << 32);
    // floor(k T / M) = k q + floor(k r / M) with q = T / M, r = T % M (k r < M^2 fits 64 bits)
    const unsigned long long um = (unsigned long long)M, q = T / um, rm = T % um;
    const unsigned long long uk = (unsigned long long)k;
    const unsigned long long lo = uk * q + (uk * rm) / um;
    const unsigned long long hi = (uk + 1) * q + ((uk + 1) * rm) / um;
    const unsigned long long width = hi - lo;
    P.valid = width != 0;
    if (!P.valid) return;   // same for both lanes of the pair
    const U64x4 r = philox4x64(uk, 0, c2, iter, a.seed, 0);
    const unsigned long long target = lo + __umul64hi(r.x[0], width);
    int elo = 0, ehi = E - 1;   // first e with cdf[e] > target
    while (elo < ehi) {
        int mid = (elo + ehi) >> 1;
        if (cdf[mid] > target) ehi = mid; else elo = mid + 1;
    }
    const int e = elo;
    P.e = e;
    const EdgeRec qe = rec[e];
    const float u = u24_hi(r.x[1]);
    const float t = qe.t0 + u * (qe.t1 - qe.t0);
    const float dx = qe.bx - qe.ax, dy = qe.by - qe.ay;
    const float x = qe.ax + t * dx;
    const float y = qe.ay + t * dy;
    const float len = sqrtf(dx * dx + dy * dy);
    P.t = t;
    P.nhx = dy / len;
    P.nhy = -dx / len;
    P.xs = side == 0 ? x + a.delta * P.nhx : x - a.delta * P.nhx;
    P.ys = side == 0 ? y + a.delta * P.nhy : y - a.delta * P.nhy;
    int px = (int)floorf(x), py = (int)floorf(y);
    px = min(max(px, 0), c.W - 1);
    py = min(max(py, 0), c.H - 1);
    P.pg = c.pix0 + (long long)py * c.W + px;
    // weight: (stratum probability width/T) / (density (wq_e/T)/len per unit length),
    // the clipped length taken in float64 with the contribution
    P.wgt = (float)width / (float)qe.wq;
}

// Closest hit and colour of this lane's side point of sample P.
template <bool COUNT>
__device__ __forceinline__ void edge_side_colour(const EdgeArgs& a, const EdgePoint& P, int* wst,
                                                 TraceCount& tc, unsigned long long& n_rays,
                                                 unsigned long long& n_hit, float col[3])
{
    const ViewDev& c = a.views[P.vi];
    const int hand = c.hand;
    const Node* nodes = a.nodes + (size_t)hand * a.n_nodes;
    const Tri* tris = a.tris + (size_t)hand * a.m.F;
    const float* normals = a.normals + (size_t)hand * a.m.V * 3;
    const float* tex = a.albedo + (size_t)hand * a.tex_h * a.tex_w * 3;
    const float bg[3] = {a.background[3 * P.pg], a.background[3 * P.pg + 1], a.background[3 * P.pg + 2]};
    Ray ray;
    Hit h;
    ray_screen(c, P.xs, P.ys, ray);
    // the wave traverses as one packet (the side points are spread along
    // silhouettes, over many screen bins); lanes of several hands (at the
    // hands' boundaries in the sample order) take one packet per hand, the
    // other lanes inactive
    if (__all(hand == __builtin_amdgcn_readfirstlane(hand))) {
        trace_wave<COUNT, true>(nodes, tris, ray, true, wst, h, &tc);
    } else {
        h.face = -1;
        h.slot = 0;
        h.t = 0.0f;
        uint64_t todo = wave_mask(true);
        while (todo) {
            const int hl = __builtin_amdgcn_readlane(hand, __ffsll((long long)todo) - 1);
            const bool mine = hand == hl;
            todo &= ~wave_mask(mine);
            Hit hh;
            trace_wave<COUNT, true>(a.nodes + (size_t)hl * a.n_nodes, a.tris + (size_t)hl * a.m.F, ray, mine, wst,
                                    hh, &tc);
            if (mine) h = hh;
        }
    }
    if (COUNT) { ++n_rays; n_hit += h.face >= 0; }
    shade_or_bg(h, tris, c, P.xs, P.ys, normals, a.uv, tex, a.tex_h, a.tex_w, a.shading, bg, col);
}

// Boundary contribution of one sample: pixel gradient g, colour step
// dc = c(x - delta n) - c(x + delta n); statistics for the proposal; the
// vertex-gradient atomics.
__device__ __forceinline__ void edge_contribution(const EdgeArgs& a, int vi, int e, float t, float wgt,
                                                  long long pg, const float dc[3])
{
    const int E = a.m.E;
    const float g[3] = {a.dimage[3 * pg], a.dimage[3 * pg + 1], a.dimage[3 * pg + 2]};
    if (g[0] == 0.0f && g[1] == 0.0f && g[2] == 0.0f) return;
    float* dcs = a.stat_dc ? a.stat_dc + ((size_t)vi * E + e) * 4 : nullptr;
    if (dcs) {   // colour-jump statistics of the edge (proposal features)
        unsafeAtomicAdd(dcs + 0, fabsf(dc[0]));
        unsafeAtomicAdd(dcs + 1, fabsf(dc[1]));
        unsafeAtomicAdd(dcs + 2, fabsf(dc[2]));
        unsafeAtomicAdd(dcs + 3, 1.0f);
    }
    const double jump = (double)g[0] * dc[0] + (double)g[1] * dc[1] + (double)g[2] * dc[2];
    if (jump == 0.0) return;
    const ViewDev& c = a.views[vi];
    const EdgeRec qe = a.rec[(size_t)vi * E + e];
    const int va = a.m.edges[2 * e], vb = a.m.edges[2 * e + 1];
    const float* vh = a.verts + (size_t)c.hand * a.m.V * 3;
    // the edge's screen normal, clipped length and projection Jacobians in
    // float64 from the float32 vertices (the float32 endpoints of the edge
    // record only placed the sample)
    double pa[2], pb[2], Ja[2][3], Jb[2][3];
    project64(c, vh + 3 * va, pa, Ja);
    project64(c, vh + 3 * vb, pb, Jb);
    const double dx = pb[0] - pa[0], dy = pb[1] - pa[1];
    const double len = sqrt(dx * dx + dy * dy);
    const double nhx = dy / len, nhy = -dx / len;
    const double sc = jump * (len * ((double)qe.t1 - (double)qe.t0)) * (double)wgt;
    if (a.stat_a) unsafeAtomicAdd(a.stat_a + (size_t)vi * E + e, (float)fabs(sc));
    // one slot array per view: the samples of a view share few vertices, so
    // the memory-side atomics of different views never queue on one address;
    // float64 sums (a vertex's samples come with both signs)
    double* gout = reinterpret_cast<double*>(a.gacc) + (size_t)vi * a.m.V * 3;
    const double sa = (1.0 - (double)t) * sc, sb = (double)t * sc;
    for (int k3 = 0; k3 < 3; ++k3) {
        unsafeAtomicAdd(gout + 3 * va + k3, sa * (Ja[0][k3] * nhx + Ja[1][k3] * nhy));
        unsafeAtomicAdd(gout + 3 * vb + k3, sb * (Jb[0][k3] * nhx + Jb[1][k3] * nhy));
    }
}

// Edge samples, one per lane pair (the even lane traces x + delta n, the odd
// lane x - delta n; consecutive global indices are consecutive strata of one
// view's CDF).  This lane pair takes samples first, first + npairs, ...
//   TRACE: samples kg < min(total, cap): trace and shade both side points
//          (independent of the image gradient) and store the sample record;
//   WEIGH: samples kg < min(total, cap) from their records, the samples
//          beyond the capacity traced in place; contributions added.
enum EdgeMode { kEdgeTrace = 0, kEdgeWeigh = 1 };

template <bool COUNT, int MODE>
__device__ void edge_samples(const EdgeArgs& a, long long first, long long npairs, int* wstack)
{
    const uint64_t iter = iteration(a.iter_dev, a.iter);
    int* wst = wstack + kMaxStack * (threadIdx.x >> 6);
    const long long total = a.prefix[a.n_views];
    const long long stored = min(total, a.sample_cap);
    const int side = threadIdx.x & 1;
    TraceCount tc;
    unsigned long long n_rays = 0, n_hit = 0;
    if (MODE == kEdgeTrace) {
        for (long long kg = first; kg < stored; kg += npairs) {
            EdgePoint P;
            edge_point(a, kg, iter, side, P);
            EdgeSample& out = a.samples[kg];
            if (!P.valid) {
                if (side == 0) out.vi = -1;
                continue;   // same for both lanes of the pair
            }
            // the record's geometry first: none of it is live across the trace
            if (side == 0) {
                out.vi = P.vi;
                out.e = P.e;
                out.pg = P.pg;
                out.t = P.t;
                out.wgt = P.wgt;
            }
            float col[3];
            edge_side_colour<COUNT>(a, P, wst, tc, n_rays, n_hit, col);
            const float o0 = __shfl_xor(col[0], 1), o1 = __shfl_xor(col[1], 1), o2 = __shfl_xor(col[2], 1);
            if (side != 0) continue;
            out.dc[0] = o0 - col[0];   // c(x - delta n) - c(x + delta n)
            out.dc[1] = o1 - col[1];
            out.dc[2] = o2 - col[2];
        }
    } else {
        for (long long kg = first; kg < stored; kg += npairs) {
            if (side != 0) continue;
            const EdgeSample rs = a.samples[kg];
            if (rs.vi < 0) continue;
            edge_contribution(a, rs.vi, rs.e, rs.t, rs.wgt, rs.pg, rs.dc);
        }
        for (long long kg = stored + first; kg < total; kg += npairs) {
            EdgePoint P;
            edge_point(a, kg, iter, side, P);
            if (!P.valid) continue;   // same for both lanes of the pair
            const float* gp = a.dimage + 3 * P.pg;
            if (gp[0] == 0.0f && gp[1] == 0.0f && gp[2] == 0.0f) continue;   // same for both lanes
            float col[3];
            edge_side_colour<COUNT>(a, P, wst, tc, n_rays, n_hit, col);
            const float o0 = __shfl_xor(col[0], 1), o1 = __shfl_xor(col[1], 1), o2 = __shfl_xor(col[2], 1);
            if (side != 0) continue;
            const float dc[3] = {o0 - col[0], o1 - col[1], o2 - col[2]};
            edge_contribution(a, P.vi, P.e, P.t, P.wgt, P.pg, dc);
        }
    }
    if (COUNT) {
        atomicAdd(a.counts + 0, n_rays);
        atomicAdd(a.counts + 1, (unsigned long long)tc.nodes);
        atomicAdd(a.counts + 2, (unsigned long long)tc.tris);
        atomicAdd(a.counts + 3, n_hit);
        atomicAdd(a.counts + 4, (unsigned long long)tc.nodes_w);
        atomicAdd(a.counts + 5, (unsigned long long)tc.tris_w);
    }
}

// ===========================================================================
// launches of the ray-tracing work
// ===========================================================================

// The few-tile render's edge waves: a wave takes pw lane pairs (one sample
// per pair), 32 while the samples are many; when they are few, smaller
// packets (down to 2 pairs) give more and shorter chains (an incoherent
// packet walks the union of its rays' paths), as long as the edge waves stay
// at most one per compute unit.  Returns their number (at most half the waves).
__device__ __forceinline__ int edge_waves_adaptive(const EdgeArgs& e, int with_edges, int nw, int& pw)
{
    pw = 32;
    if (!with_edges) return 0;
    const long long stored = min(e.prefix[e.n_views], e.sample_cap);
    while (pw > 2 && (stored + pw / 2 - 1) / (pw / 2) <= e.few_waves) pw >>= 1;
    return (int)min((stored + pw - 1) / pw, (long long)max(1, nw / 2));
}

template <bool COUNT>
__device__ __forceinline__ void render_edge_wave(const EdgeArgs& e, int gw, int n_ew, int pw, int* wstack)
{
    const int pr = (threadIdx.x & 63) >> 1;   // the lane's pair; pairs past pw idle
    const long long first = pr < pw ? (long long)gw * pw + pr : (1LL << 62);
    edge_samples<COUNT, kEdgeTrace>(e, first, (long long)n_ew * pw, wstack);
}

// Render: every block writes its share of the pixels outside the views'
// tiled rectangles; with edges, the first waves trace the edge samples' side
// points (a wave packet per hand the wave's samples look at) while the
// others render the wave tiles (one traversal stack per wave).
template <bool COUNT, bool RASTER>
__global__ void __launch_bounds__(kThreads, 5) k_render(RenderArgs a, EdgeArgs e, int with_edges)
{
    __shared__ int wstack[kMaxStack * (kThreads / 64)];
    const int bid = (int)blockIdx.x, nb = (int)gridDim.x;
    render_side_work(a, bid, nb);
    if (a.hit_iter && bid == 0 && threadIdx.x == 0) *a.hit_iter = (int)iteration(a.iter_dev, a.iter);
    const int gw = __builtin_amdgcn_readfirstlane((int)((bid * kThreads + threadIdx.x) >> 6));
    const int nw = (int)((nb * kThreads) >> 6);
    // the first n_ew waves trace the edge samples (32 lane pairs each), from
    // the start: their traversals are long dependent chains; the other waves
    // render the tiles.  (The few-tile render's adaptive packet size costs
    // this kernel's tile path scalar registers and time.)
    int n_ew = 0;
    if (with_edges) {
        const long long stored = min(e.prefix[e.n_views], e.sample_cap);
        n_ew = (int)min((stored + 31) / 32, (long long)max(1, nw / 2));
    }
    if (gw < n_ew) {
        const long long first = (long long)gw * 32 + ((threadIdx.x & 63) >> 1);
        edge_samples<COUNT, kEdgeTrace>(e, first, (long long)n_ew * 32, wstack);
    } else {
        render_tiles<COUNT, RASTER>(a, gw - n_ew, nw - n_ew, wstack);
    }
}

// The same render for scenes with few tiles (the tiles of all views at most
// one per SIMD, ray tracing only; grid of at least two blocks): most SIMDs
// would idle, and a tile's bin walk is one wave's chain of triangle tests,
// so the waves of a block share each tile (render_tiles with SPLIT); the
// edge waves take whole blocks, leaving at least one block to the tiles.
template <bool COUNT>
__global__ void __launch_bounds__(kThreads, 5) k_render_few(RenderArgs a, EdgeArgs e, int with_edges)
{
    constexpr int kSplit = kThreads / 64;
    __shared__ int wstack[kMaxStack * kSplit];
    __shared__ float xch[2 * kThreads * 3];   // the waves' partial hits
    const int bid = (int)blockIdx.x, nb = (int)gridDim.x;
    render_side_work(a, bid, nb);
    if (a.hit_iter && bid == 0 && threadIdx.x == 0) *a.hit_iter = (int)iteration(a.iter_dev, a.iter);
    const int gw = __builtin_amdgcn_readfirstlane((int)((bid * kThreads + threadIdx.x) >> 6));
    const int nw = (int)((nb * kThreads) >> 6);
    int pw;
    int n_ew = edge_waves_adaptive(e, with_edges, nw, pw);
    n_ew = min((n_ew + kSplit - 1) / kSplit * kSplit, (nb - 1) * kSplit);
    if (gw < n_ew)
        render_edge_wave<COUNT>(e, gw, n_ew, pw, wstack);
    else
        render_tiles<COUNT, false, kSplit>(a, bid - n_ew / kSplit, nb - n_ew / kSplit, wstack, xch);
}

// Edge samples, first part: trace and shade both side points of every stored
// sample (needs only the geometry and the silhouette tables).
template <bool COUNT>
__global__ void __launch_bounds__(kThreads) k_edge_trace(EdgeArgs e)
{
    __shared__ int wstack[kMaxStack * (kThreads / 64)];
    edge_samples<COUNT, kEdgeTrace>(e, ((long long)blockIdx.x * kThreads + threadIdx.x) >> 1,
                                    ((long long)gridDim.x * kThreads) >> 1, wstack);
}

// Backward ray tracing: the first `n_edge` blocks draw the edge samples, the
// rest run the interior adjoint; in one launch the latency-bound edge
// samples overlap with the adjoint's arithmetic.
template <bool COUNT>
__global__ void __launch_bounds__(kThreads) k_backward_trace(AdjointArgs a, EdgeArgs e, int n_edge, LossArgs l,
                                                             int n_loss)
{
    // adjoint blocks: the texel windows of their waves
    __shared__ __align__(16) int lds[kWaveWin * (kThreads / 64)];
    __shared__ float stage[64 * kStageW * (kThreads / 64)];   // adjoint blocks: staged texel scatters
    __shared__ int wstack[kMaxStack * (kThreads / 64)];
    if ((int)blockIdx.x < n_edge) {
        edge_samples<COUNT, kEdgeWeigh>(e, ((long long)blockIdx.x * kThreads + threadIdx.x) >> 1,
                                        ((long long)n_edge * kThreads) >> 1, wstack);
        return;
    }
    // the last n_loss blocks: partial sums of the loss value (chunk per block)
    const int n_adj = (int)gridDim.x - n_edge - n_loss;
    if ((int)blockIdx.x >= n_edge + n_adj) {
        loss_partial(l, (int)blockIdx.x - n_edge - n_adj);
        return;
    }
    adjoint_tiles<COUNT>(a, (int)blockIdx.x - n_edge, n_adj, wstack, reinterpret_cast<float*>(lds), stage);
}

// ===========================================================================
// geometry backward: normals, skinning, joint tree (one block per hand)
// ===========================================================================

// The sums over the vertices (`tot`: global rotation and translation, per
// joint dL/dGR_j and dL/dAt_j, shape) taken through the joint tree, one level
// at a time from the leaves, and the Rodrigues maps to dL/dparams.  The first
// wave does the work, lane j for joint j; the caller's next block barrier
// orders its results for the other waves.
// What lane j of the finish reads from global memory, loaded ahead (the
// finish runs in whichever block of the hand ends last): rows j and j + 64
// of J_reg S (joint coordinate row / 3, row % 3 per shape coefficient) for
// the shape gradient, the lane's rotation parameters, its joint's depth and
// parent.
struct FinishIn {
    float jsr[2][kMaxShape];
    float r[3];
    int dj, par;
};

__device__ __forceinline__ void finish_load(const MeshDev& m, const float* __restrict__ p, FinishIn& in)
{
    const int J = m.J, K = m.K;
    const int j = threadIdx.x & 63;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k = 0; k < kMaxShape; ++k) {
            const int row = min(j + 64 * h, 3 * J - 1), kk = k < K ? k : K - 1;
            in.jsr[h][k] = K > 0 && J > 0 ? m.js[row * K + kk] : 0.0f;
        }
    const float* pr = j < J ? p + 3 * j : p + 58;
    for (int c = 0; c < 3; ++c) in.r[c] = pr[c];
    in.dj = j < J ? m.jdepth[j] : -1;
    in.par = j < J ? m.parents[j] : -1;
}

__device__ void skin_bwd_finish(const MeshDev& m, const FinishIn& in, const float* tot, const JointState& js,
                                float* __restrict__ gp, const float* xGt)
{
    __shared__ float gJs[kMaxJoints * 3];   // dL/dJ for the shape rows at the end
    const int J = m.J, K = m.K;
    const int j = threadIdx.x;
    if (j >= 64) return;
    const float* r = in.r;
    const int dj = in.dj, par = in.par;
    // children of joint j (bit c: joint c), from the parents' lanes
    unsigned int kids = 0u;
    for (int c = 0; c < J; ++c)
        if (__builtin_amdgcn_readlane(par, c) == j) kids |= 1u << c;
    // the joint's state, read once: GR_j, GR_parent, R_j, J_j - J_parent
    const int jl = j < J ? j : 0, pl = par >= 0 ? par : 0;
    float GRj[9], GRp[9], Rc[9], d[3];
    for (int i = 0; i < 9; ++i) {
        GRj[i] = js.GR[9 * jl + i];
        GRp[i] = js.GR[9 * pl + i];
        Rc[i] = js.rod[jl].R[i];
    }
    for (int i = 0; i < 3; ++i) d[i] = js.J[3 * jl + i] - js.J[3 * pl + i];
    // At_j = Gt_j - GR_j J_j
    float gGR[9], gGt[3], gJ[3];
    {
        const float* a = tot + 12 + 12 * jl;
        for (int i = 0; i < 3; ++i) {
            gGt[i] = a[9 + i] + (xGt ? xGt[3 * jl + i] : 0.0f);
            for (int k = 0; k < 3; ++k) gGR[3 * i + k] = a[3 * i + k] - a[9 + i] * js.J[3 * jl + k];
        }
        float y[3];
        matTvec3(GRj, a + 9, y);
        for (int i = 0; i < 3; ++i) gJ[i] = -y[i];
    }
    // Gt_j = GR_p (J_j - J_p) + Gt_p, GR_j = GR_p R_j: the joints of level L
    // finish their own terms and leave those of their parent in registers;
    // the parents (level L - 1) read them from the children's lanes and add
    // them in child order.  Every value stays in its lane's registers.
    float gR[9], cGR[9], cJ[3];
    for (int i = 0; i < 9; ++i) gR[i] = cGR[i] = 0.0f;
    for (int i = 0; i < 3; ++i) cJ[i] = 0.0f;
    for (int L = m.max_depth; L >= 0; --L) {
        if (dj == L) {
            if (par < 0) {
                for (int i = 0; i < 9; ++i) gR[i] = gGR[i];
                for (int i = 0; i < 3; ++i) gJ[i] = gJ[i] + gGt[i];
            } else {
                float y[3];
                matTvec3(GRp, gGt, y);
                for (int i = 0; i < 3; ++i) {
                    gJ[i] = gJ[i] + y[i];
                    cJ[i] = y[i];
                }
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 3; ++k) {
                        float s = 0.0f;
                        for (int q = 0; q < 3; ++q) s += GRp[3 * q + i] * gGR[3 * q + k];
                        gR[3 * i + k] = s;
                    }
                for (int i = 0; i < 3; ++i)
                    for (int k = 0; k < 3; ++k) {
                        float s = gGt[i] * d[k];
                        for (int q = 0; q < 3; ++q) s += gGR[3 * i + q] * Rc[3 * k + q];
                        cGR[3 * i + k] = s;
                    }
            }
        }
        // the parents of level L - 1: one child per round (the loop and its
        // lane reads run on the whole wave)
        unsigned int rem = j < J && dj == L - 1 ? kids : 0u;
        while (__any(rem != 0u)) {
            const int c = rem ? __builtin_ctz(rem) : j;
            float xGR[9], xJ[3], xT[3];
            for (int i = 0; i < 9; ++i) xGR[i] = __shfl(cGR[i], c);
            for (int i = 0; i < 3; ++i) {
                xJ[i] = __shfl(cJ[i], c);
                xT[i] = __shfl(gGt[i], c);
            }
            if (rem) {
                for (int i = 0; i < 9; ++i) gGR[i] += xGR[i];
                for (int i = 0; i < 3; ++i) {
                    gJ[i] -= xJ[i];
                    gGt[i] += xT[i];
                }
                rem &= rem - 1u;
            }
        }
    }
    if (j < J) rodrigues_bwd(r, js.rod[j], gR, gp + 3 * j);
    if (j == J) rodrigues_bwd(r, js.rod[J], tot, gp + 58);
    for (int q = J + j; q < 16; q += 64) gp[3 * q] = gp[3 * q + 1] = gp[3 * q + 2] = 0.0f;
    if (j < 3) gp[61 + j] = tot[9 + j];
    // shape: vertex part + joint part (J = J_reg T + (J_reg S) beta), the
    // joint part as lane j's row times dL/dJ[j], summed over the wave
    if (j < J)
        for (int i = 0; i < 3; ++i) gJs[3 * j + i] = gJ[i];
    wave_lds_sync();
    float sj[kMaxShape];
    const float gj0 = j < 3 * J ? gJs[j] : 0.0f, gj1 = j + 64 < 3 * J ? gJs[j + 64] : 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxShape; ++k) sj[k] = in.jsr[0][k] * gj0 + in.jsr[1][k] * gj1;
    wave_sum63_n<kMaxShape>(sj);
    if (j == 63)
#pragma unroll
        for (int k = 0; k < 10; ++k) gp[48 + k] = k < K ? tot[12 + 12 * J + k] + sj[k] : 0.0f;
}

// Joint prior (Section 3.2, Eq. 5): lambda times the coordinate-wise smooth L1
// distance, with threshold gamma, between the posed joints Rp Gt_j + tau and
// the target joints (quadratic d^2 / (2 gamma) below gamma, |d| - gamma / 2
// above).  One wave, lane j for joint j.  Its gradient g_j with respect to the
// posed joint enters the global rotation and translation sums (tot[0..8] as
// g_j Gt_j^T, tot[9..11] as g_j) and, as Rp^T g_j, dL/dGt_j (xGt, LDS);
// lambda E2 is added to *loss when it is given.
__device__ void joint_prior(const MeshDev& m, const JointState& js, const float* __restrict__ p,
                            const float* __restrict__ target, float lambda, float gamma, float* tot,
                            float* xGt, float* loss)
{
    const int j = threadIdx.x;
    float g[3] = {0.0f, 0.0f, 0.0f}, x[3] = {0.0f, 0.0f, 0.0f}, e = 0.0f;
    if (j < m.J) {
        for (int i = 0; i < 3; ++i) x[i] = js.Gt[3 * j + i];
        float y[3];
        matvec3(js.Rp, x, y);
        for (int i = 0; i < 3; ++i) {
            const float d = (y[i] + p[61 + i]) - target[3 * j + i];
            const float ad = fabsf(d);
            if (ad < gamma) {
                e += 0.5f * d * d / gamma;
                g[i] = lambda * d / gamma;
            } else {
                e += ad - 0.5f * gamma;
                g[i] = d > 0.0f ? lambda : -lambda;
            }
        }
        matTvec3(js.Rp, g, xGt + 3 * j);
    }
    float sv[13];
    for (int i = 0; i < 3; ++i) {
        for (int k = 0; k < 3; ++k) sv[3 * i + k] = g[i] * x[k];
        sv[9 + i] = g[i];
    }
    sv[12] = lambda * e;
    wave_sum63_n<13>(sv);
    if (j == 63) {
        for (int k = 0; k < 12; ++k) tot[k] += sv[k];
        if (loss) *loss += sv[12];
    }
    wave_lds_sync();
}

// One Adam update (bias corrections bc1, bc2), the arithmetic of every
// parameter and colour-map entry.
__device__ __forceinline__ float adam_update(float x, float* m, float* v, float g, float lr, const AdamArgs& a,
                                             float bc1, float bc2)
{
    const float m2 = a.beta1 * *m + (1.0f - a.beta1) * g;
    const float v2 = a.beta2 * *v + (1.0f - a.beta2) * g * g;
    *m = m2;
    *v = v2;
    const float mh = m2 / bc1, vh = v2 / bc2;
    return x - lr * mh / (sqrtf(vh) + a.eps);
}

__device__ __forceinline__ void adam_bias(const AdamArgs& a, float& bc1, float& bc2)
{
    bc1 = a.bc1;
    bc2 = a.bc2;
    if (a.iter_dev) {
        const double t = (double)(*a.iter_dev) + 1.0;
        bc1 = (float)(1.0 - pow((double)a.beta1, t));
        bc2 = (float)(1.0 - pow((double)a.beta2, t));
    }
}

__device__ __forceinline__ float param_lr(const AdamArgs& a, int k)
{
    return k < 3 ? a.lr[0] : k < 48 ? a.lr[1] : k < 58 ? a.lr[2] : k < 61 ? a.lr[3] : a.lr[4];
}

// Adam on the parameters (64 per hand) and on the colour map (clamped to
// [0, 1], four entries per step), grid-stride over thread index tid of n.
__device__ __forceinline__ void adam_params_part(const AdamArgs& a, float bc1, float bc2, long long tid,
                                                 long long stride)
{
    const long long np = 64ll * a.n_hands;
    for (long long i = tid; i < np; i += stride) {
        const float lr = param_lr(a, (int)(i % 64));
        if (lr != 0.0f)
            a.params[i] = adam_update(a.params[i], a.m_params + i, a.v_params + i, a.grad_params[i], lr, a, bc1, bc2);
    }
}

__device__ __forceinline__ void adam_albedo_part(const AdamArgs& a, float bc1, float bc2, long long tid,
                                                 long long stride)
{
    const float lr = a.lr[5];
    if (lr == 0.0f) return;
    const long long n4 = a.n_albedo >> 2;
    float4* x4 = reinterpret_cast<float4*>(a.albedo);
    float4* m4 = reinterpret_cast<float4*>(a.m_albedo);
    float4* v4 = reinterpret_cast<float4*>(a.v_albedo);
    const float4* g4 = reinterpret_cast<const float4*>(a.grad_albedo);
    for (long long q = tid; q < n4; q += stride) {
        float4 x = x4[q], mm = m4[q], vv = v4[q];
        const float4 g = g4[q];
        x.x = fminf(fmaxf(adam_update(x.x, &mm.x, &vv.x, g.x, lr, a, bc1, bc2), 0.0f), 1.0f);
        x.y = fminf(fmaxf(adam_update(x.y, &mm.y, &vv.y, g.y, lr, a, bc1, bc2), 0.0f), 1.0f);
        x.z = fminf(fmaxf(adam_update(x.z, &mm.z, &vv.z, g.z, lr, a, bc1, bc2), 0.0f), 1.0f);
        x.w = fminf(fmaxf(adam_update(x.w, &mm.w, &vv.w, g.w, lr, a, bc1, bc2), 0.0f), 1.0f);
        x4[q] = x; m4[q] = mm; v4[q] = vv;
    }
    for (long long j = 4 * n4 + tid; j < a.n_albedo; j += stride)
        a.albedo[j] = fminf(fmaxf(adam_update(a.albedo[j], a.m_albedo + j, a.v_albedo + j, a.grad_albedo[j], lr, a,
                                              bc1, bc2), 0.0f), 1.0f);
}


// Geometry backward in two launches.
//
// k_geom_p1, grid (vertex blocks, hands): per vertex, its own slot and the
// triangle-corner slots it occupies (position and normal parts), the raw
// normal s (the forward's face cross products in the same order) and the
// normalisation backward dL/ds = (gn - (gn . n) n) / |s|.  The block past
// the vertex blocks sums the hand's loss value from the chunk partials.
__global__ void __launch_bounds__(256) k_geom_p1(GeomBwdArgs a)
{
    const MeshDev& m = a.m;
    const int V = m.V;
    // blocks [0, H * per_hand): per hand, vertex blocks and the loss block;
    // the rest: the colour map's Adam step (with adam_albedo)
    const int per_hand = a.p1_blocks + 1;
    const int bid = blockIdx.x;
    if (bid >= a.n_hands * per_hand) {
        float bc1, bc2;
        adam_bias(a.adam, bc1, bc2);
        const long long nb = (long long)gridDim.x - (long long)a.n_hands * per_hand;
        adam_albedo_part(a.adam, bc1, bc2, (long long)(bid - a.n_hands * per_hand) * blockDim.x + threadIdx.x,
                         nb * blockDim.x);
        return;
    }
    const int h = bid / per_hand, bx = bid - h * per_hand;
    if (bx == a.p1_blocks) {
        if (a.with_loss) loss_value_hand(a.loss, h);
        return;
    }
    const int v = bx * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float* vh = a.verts + (size_t)h * V * 3;
    const float* gf = a.gface + (size_t)h * m.F * 18;
    // the edge term's float64 slots of the hand's views, in view order; the
    // sums of the vertex run in float64
    double g[3] = {0.0, 0.0, 0.0}, gn[3] = {0.0, 0.0, 0.0};
    for (int q = a.hand_view_off[h]; q < a.hand_view_off[h + 1]; ++q) {
        const double* ga = reinterpret_cast<const double*>(a.gacc) + ((size_t)a.hand_views[q] * V + v) * 3;
        for (int k = 0; k < 3; ++k) g[k] += ga[k];
    }
    float sv[3] = {0.0f, 0.0f, 0.0f};
    // faces around v: the corner table's entries with all their loads in
    // flight, then any faces beyond it from the CSR list, in list order
    const int k0 = m.vf_off[v], k1 = m.vf_off[v + 1];
    int4 cq[kVfSlots];
#pragma unroll
    for (int k = 0; k < kVfSlots; ++k) cq[k] = m.vf_corner[(size_t)k * V + v];
    auto face_terms = [&](int f, int i0, int i1, int i2) {
        const int corner = i0 == v ? 0 : (i1 == v ? 1 : 2);
        const float* sl = gf + 18 * f + 6 * corner;
        for (int q = 0; q < 3; ++q) { g[q] += (double)sl[q]; gn[q] += (double)sl[3 + q]; }
        const float* a0 = vh + 3 * i0;
        const float* a1 = vh + 3 * i1;
        const float* a2 = vh + 3 * i2;
        const float e1[3] = {a1[0] - a0[0], a1[1] - a0[1], a1[2] - a0[2]};
        const float e2[3] = {a2[0] - a0[0], a2[1] - a0[1], a2[2] - a0[2]};
        sv[0] += e1[1] * e2[2] - e1[2] * e2[1];
        sv[1] += e1[2] * e2[0] - e1[0] * e2[2];
        sv[2] += e1[0] * e2[1] - e1[1] * e2[0];
    };
#pragma unroll
    for (int k = 0; k < kVfSlots; ++k)
        if (k < k1 - k0) face_terms(cq[k].w, cq[k].x, cq[k].y, cq[k].z);
    for (int k = k0 + kVfSlots; k < k1; ++k) {
        const int f = m.vf_faces[k];
        face_terms(f, m.faces[3 * f], m.faces[3 * f + 1], m.faces[3 * f + 2]);
    }
    const float il = 1.0f / sqrtf(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]);
    const float n[3] = {sv[0] * il, sv[1] * il, sv[2] * il};
    const float gnf[3] = {(float)gn[0], (float)gn[1], (float)gn[2]};
    if (a.grad_normals) {
        float* o = a.grad_normals + ((size_t)h * V + v) * 3;
        o[0] = gnf[0]; o[1] = gnf[1]; o[2] = gnf[2];
    }
    const float d = gnf[0] * n[0] + gnf[1] * n[1] + gnf[2] * n[2];
    float* gr = a.gr + ((size_t)h * V + v) * 3;
    float* gp = a.gpos + ((size_t)h * V + v) * 3;
    for (int q = 0; q < 3; ++q) {
        gr[q] = (gnf[q] - d * n[q]) * il;
        gp[q] = (float)g[q];
    }
}

// k_geom_p2, grid (vertex blocks of one wave, hands): the raw normals'
// gradient to the vertices through the face cross products, dL/dv, then the
// skinning backward with the block's sums (DPP wave sums) written as one
// row of partials; the last block of the hand adds the rows in block order,
// takes them through the joint tree and, with adam_params, steps the
// parameters.
// Gradient at vertex v (a corner of face (ia, ib, ic)) of the face's raw
// normal (b - a) x (c - a), given dL/d(raw face normal) as the sum of its
// corners' raw-vertex-normal gradients.  A face (v, v, v) adds exact zeros.
__device__ __forceinline__ void normal_corner_grad(int v, int ia, int ib, int ic, const float* __restrict__ vh,
                                                   const float* __restrict__ grh, float* g)
{
    float gfs[3];
    for (int q = 0; q < 3; ++q) gfs[q] = grh[3 * ia + q] + grh[3 * ib + q] + grh[3 * ic + q];
    const float e1[3] = {vh[3 * ib] - vh[3 * ia], vh[3 * ib + 1] - vh[3 * ia + 1], vh[3 * ib + 2] - vh[3 * ia + 2]};
    const float e2[3] = {vh[3 * ic] - vh[3 * ia], vh[3 * ic + 1] - vh[3 * ia + 1], vh[3 * ic + 2] - vh[3 * ia + 2]};
    const float g1[3] = {e2[1] * gfs[2] - e2[2] * gfs[1], e2[2] * gfs[0] - e2[0] * gfs[2],
                         e2[0] * gfs[1] - e2[1] * gfs[0]};
    const float g2[3] = {gfs[1] * e1[2] - gfs[2] * e1[1], gfs[2] * e1[0] - gfs[0] * e1[2],
                         gfs[0] * e1[1] - gfs[1] * e1[0]};
    for (int q = 0; q < 3; ++q) {
        const float d = v == ia ? -(g1[q] + g2[q]) : (v == ib ? g1[q] : g2[q]);
        g[q] += d;
    }
}

__global__ void __launch_bounds__(64) k_geom_p2(GeomBwdArgs a)
{
    __shared__ JointState js;
    __shared__ float acc[kSkinPart];
    __shared__ int last;
    const MeshDev& m = a.m;
    const int h = blockIdx.y, t = threadIdx.x;
    const int V = m.V, J = m.J, K = m.K;
    const int n_part = 12 + 12 * J + K;
    const float* p = a.params + 64 * h;
    const int v = blockIdx.x * 64 + t;
    // the vertex's tables first: their loads are in flight with the joint
    // state's
    float tpl[3] = {0.0f, 0.0f, 0.0f}, sd[3][kMaxShape] = {}, wq[kMaxInfl] = {};
    int jq[kMaxInfl] = {};
    if (v < V) {
        load_weights(m, v, wq, jq);
        load_shape(m, v, tpl, sd);
    }
    for (int i = t; i < n_part; i += 64) acc[i] = 0.0f;
    // the finish's reads and the parameters' Adam state, in case this block
    // ends last
    FinishIn fin;
    finish_load(m, p, fin);
    float ax = 0.0f, am = 0.0f, av = 0.0f;
    if (a.adam_params) {
        const size_t i = (size_t)64 * h + t;
        ax = a.adam.params[i];
        am = a.adam.m_params[i];
        av = a.adam.v_params[i];
    }
    if (a.js_saved) {
        // the skinning launch of these parameters left the joint state
        const float* src = a.js_saved + (size_t)h * kJointStateFloats;
        float* dst = reinterpret_cast<float*>(&js);
        constexpr int kPer = (kJointStateFloats + 63) / 64;
        float x[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) x[q] = src[min(t + 64 * q, kJointStateFloats - 1)];
#pragma unroll
        for (int q = 0; q < kPer; ++q)
            if (t + 64 * q < kJointStateFloats) dst[t + 64 * q] = x[q];
        __syncthreads();
    } else {
        joint_state(m, p, js);   // ends with a barrier
    }
    const float* vh = a.verts + (size_t)h * V * 3;
    const float* grh = a.gr + (size_t)h * V * 3;
    float bk[kMaxShape];
    load_beta(m, p + 48, bk);
    float g[3] = {0.0f, 0.0f, 0.0f}, x[3] = {0.0f, 0.0f, 0.0f}, vp[3] = {0.0f, 0.0f, 0.0f};
    float gvp[3] = {0.0f, 0.0f, 0.0f}, gx[3] = {0.0f, 0.0f, 0.0f};
    unsigned int jmask = 0u;   // joints this vertex is bound to
    if (v < V) {
        shape_vertex(m, bk, tpl, sd, x);
        for (int q = 0; q < 3; ++q) g[q] = a.gpos[((size_t)h * V + v) * 3 + q];
        // faces around v: the padded corner table with all its loads in
        // flight together, then the faces beyond it (rare) from the CSR list
        const int k0 = m.vf_off[v], k1 = m.vf_off[v + 1];
        int4 cq[kVfSlots];
#pragma unroll
        for (int k = 0; k < kVfSlots; ++k) cq[k] = m.vf_corner[(size_t)k * V + v];
#pragma unroll
        for (int k = 0; k < kVfSlots; ++k)
            if (k < k1 - k0) normal_corner_grad(v, cq[k].x, cq[k].y, cq[k].z, vh, grh, g);
        for (int k = k0 + kVfSlots; k < k1; ++k) {
            const int f = m.vf_faces[k];
            normal_corner_grad(v, m.faces[3 * f], m.faces[3 * f + 1], m.faces[3 * f + 2], vh, grh, g);
        }
        if (a.grad_verts) {
            float* o = a.grad_verts + ((size_t)h * V + v) * 3;
            o[0] = g[0]; o[1] = g[1]; o[2] = g[2];
        }
        blend_vertex(js, wq, jq, x, vp);
        matTvec3(js.Rp, g, gvp);
#pragma unroll
        for (int q = 0; q < kMaxInfl; ++q) {
            const float w = wq[q];
            if (w == 0.0f) continue;
            const int j = jq[q];
            jmask |= 1u << j;
            float y[3];
            matTvec3(js.GR + 9 * j, gvp, y);
            for (int c = 0; c < 3; ++c) gx[c] += w * y[c];
        }
    }
    // global rotation (g vp^T) and translation (g), shape through the vertex
    // offsets: all wave sums interleaved, then stored by lane 63
    {
        float sv[12 + kMaxShape];
        for (int i = 0; i < 3; ++i) {
            for (int k = 0; k < 3; ++k) sv[3 * i + k] = g[i] * vp[k];
            sv[9 + i] = g[i];
        }
#pragma unroll
        for (int k = 0; k < kMaxShape; ++k)
            sv[12 + k] = v < V ? sd[0][k] * gx[0] + sd[1][k] * gx[1] + sd[2][k] * gx[2] : 0.0f;
        wave_sum63_n<12 + kMaxShape>(sv);
        if (t == 63) {
            for (int k = 0; k < 12; ++k) acc[k] = sv[k];
            for (int k = 0; k < kMaxShape; ++k)
                if (k < K) acc[12 + 12 * J + k] = sv[12 + k];
        }
    }
    // per joint bound to a vertex of this wave: [dL/dGR_j as w gvp x^T (9),
    // dL/dAt_j as w gvp (3)]
    unsigned int wmask = jmask;
    for (int o = 1; o < 64; o <<= 1) wmask |= __shfl_xor(wmask, o);
    wmask = __builtin_amdgcn_readfirstlane(wmask);
    for (; wmask; wmask &= wmask - 1u) {
        const int j = __builtin_ctz(wmask);
        float w = 0.0f;
        if ((jmask >> j) & 1u)
#pragma unroll
            for (int q = 0; q < kMaxInfl; ++q)
                if (q < m.infl && jq[q] == j) w += wq[q];
        float sv[12];
        for (int i = 0; i < 3; ++i) {
            const float wg = w * gvp[i];
            for (int k = 0; k < 3; ++k) sv[3 * i + k] = wg * x[k];
            sv[9 + i] = wg;
        }
        wave_sum63_n<12>(sv);
        if (t == 63)
            for (int k = 0; k < 12; ++k) acc[12 + 12 * j + k] = sv[k];
    }
    __syncthreads();
    // the hand's sums: each block adds its own (memory-side atomics), the
    // last block to finish reads them and leaves zeros
    float* sums = a.part + (size_t)h * kSkinPart;
    for (int i = t; i < n_part; i += 64)
        if (acc[i] != 0.0f) unsafeAtomicAdd(sums + i, acc[i]);
    __threadfence();
    __syncthreads();
    if (t == 0) last = atomicAdd(a.counter + h, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (t == 0) a.counter[h] = 0;
    for (int i = t; i < n_part; i += 64) {
        acc[i] = __hip_atomic_load(sums + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sums[i] = 0.0f;
    }
    __syncthreads();
    float* gp = a.grad_params + 64 * h;
    __shared__ float xGt[kMaxJoints * 3];
    if (a.prior_target)
        joint_prior(m, js, p, a.prior_target + (size_t)h * J * 3, a.prior_lambda, a.prior_gamma, acc, xGt,
                    a.with_loss && a.loss.loss ? a.loss.loss + h : nullptr);
    skin_bwd_finish(m, fin, acc, js, gp, a.prior_target ? xGt : nullptr);
    if (!a.adam_params) return;
    __syncthreads();   // the finish has read the parameters and written gp
    const float lr = param_lr(a.adam, t);
    if (lr != 0.0f) {
        float bc1, bc2;
        adam_bias(a.adam, bc1, bc2);
        const size_t i = (size_t)64 * h + t;
        a.adam.params[i] = adam_update(ax, &am, &av, gp[t], lr, a.adam, bc1, bc2);
        a.adam.m_params[i] = am;
        a.adam.v_params[i] = av;
    }
    if (!a.iter_advance) return;
    // the last hand to finish advances the iteration counter: every read of
    // it in this iteration (the Adam steps above and in the previous
    // launches) has happened
    __syncthreads();
    if (t == 0) {
        __threadfence();
        if (atomicAdd(a.hand_counter, 1) == a.n_hands - 1) {
            *a.hand_counter = 0;
            *a.iter_advance += 1;
        }
    }
}

__global__ void __launch_bounds__(256) k_adam(AdamArgs a)
{
    float bc1, bc2;
    adam_bias(a, bc1, bc2);
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    adam_params_part(a, bc1, bc2, tid, stride);
    adam_albedo_part(a, bc1, bc2, tid, stride);
}

__global__ void k_advance(int* p)
{
    if (threadIdx.x == 0) *p += 1;
}

__global__ void k_set_i32(int* p, int n, int v)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = v;
}

// ===========================================================================
// camera coverage: faces seen per view, greedy camera order
// ===========================================================================

constexpr int kCoverLdsBytes = 65536;   // bitmaps of the order kernel

// visible[v, f] = 1 when a camera sample of view v hit face f (hit_face as the
// render writes it, [pixels, spp]); grid (chunks, views), dynamic LDS: a bitmap
// of the faces (the block's hits are gathered there, then written once);
// `visible` is zero before the launch.
__global__ void __launch_bounds__(256) k_face_visibility(const ViewDev* __restrict__ views,
                                                         const int* __restrict__ hit_face, int spp, int F,
                                                         int* __restrict__ visible)
{
    extern __shared__ unsigned int bits[];
    const int nwords = (F + 31) >> 5;
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) bits[i] = 0u;
    __syncthreads();
    const ViewDev& c = views[blockIdx.y];
    const long long n = (long long)c.W * c.H * spp, first = c.pix0 * spp;
    const int* hf = hit_face + first;
    auto mark = [&](int f) {
        if (f >= 0 && f < F && !((bits[f >> 5] >> (f & 31)) & 1u)) atomicOr(bits + (f >> 5), 1u << (f & 31));
    };
    const long long stride = (long long)gridDim.x * blockDim.x;
    long long done = 0;
    if ((reinterpret_cast<uintptr_t>(hf) & 15) == 0) {
        // four ids per load
        const int4* h4 = reinterpret_cast<const int4*>(hf);
        const long long n4 = n >> 2;
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
            const int4 q = h4[i];
            mark(q.x); mark(q.y); mark(q.z); mark(q.w);
        }
        done = n4 << 2;
    }
    for (long long i = done + (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) mark(hf[i]);
    __syncthreads();
    int* out = visible + (size_t)blockIdx.y * F;
    for (int i = threadIdx.x; i < nwords; i += blockDim.x)
        for (unsigned int b = bits[i]; b; b &= b - 1u) out[32 * i + __builtin_ctz(b)] = 1;
}

// Greedy order of each hand's views by coverage (one block per hand): step k
// takes the view that adds the most faces not seen by the views taken before
// (ties: the earlier view in the hand's list); order[off + k] is its view
// index, covered[off + k] the faces seen by the first k + 1 views.  The whole
// block turns the views' face flags into LDS bitmaps (8-byte loads, many in
// flight); then one wave runs the steps: a lane per candidate view counts its
// new faces by popcounts against the seen bitmap, the wave maximum of
// (gain, earlier view) picks the view, and the seen bitmap takes its bits, with
// no block barrier inside the loop.  Dynamic LDS: the views' bitmaps, the seen
// bitmap, taken flags.
__global__ void __launch_bounds__(1024) k_camera_order(const int* __restrict__ visible,
                                                       const int* __restrict__ hand_view_off,
                                                       const int* __restrict__ hand_views, int F,
                                                       int* __restrict__ order, int* __restrict__ covered)
{
    extern __shared__ __align__(16) unsigned int cs[];
    const int h = blockIdx.x, t = threadIdx.x;
    const int off = hand_view_off[h], nv = hand_view_off[h + 1] - off;
    const int nwords = (F + 31) >> 5, nwp = (nwords + 3) & ~3;   // rows padded to 16 bytes
    unsigned int* vb = cs;                                    // [nv * nwp]
    unsigned int* seen = vb + (size_t)nv * nwp;               // [nwp]
    int* taken = reinterpret_cast<int*>(seen + nwp);          // [nv]
    // word wd of view c: faces 32 wd .. 32 wd + 31, read as pairs (a view's
    // row starts at a multiple of 8 bytes when F is even; odd F reads singles)
    for (int i = t; i < nv * nwp; i += blockDim.x) {
        const int c = i / nwp, wd = i - c * nwp;
        unsigned int m = 0u;
        if (wd < nwords) {
            const int* v = visible + (size_t)hand_views[off + c] * F + 32 * wd;
            const int nb = min(32, F - 32 * wd);
            if ((F & 1) == 0 && nb == 32) {
                int2 q[16];
#pragma unroll
                for (int b = 0; b < 16; ++b) q[b] = reinterpret_cast<const int2*>(v)[b];
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    m |= (q[b].x != 0 ? 1u : 0u) << (2 * b) | (q[b].y != 0 ? 1u : 0u) << (2 * b + 1);
            } else {
                for (int b = 0; b < nb; ++b) m |= (v[b] != 0 ? 1u : 0u) << b;
            }
        }
        vb[i] = m;
    }
    for (int i = t; i < nwp; i += blockDim.x) seen[i] = 0u;
    for (int i = t; i < nv; i += blockDim.x) taken[i] = 0;
    __syncthreads();
    if (t >= 64) return;   // one wave from here on
    const int lane = t;
    const uint4* vb4 = reinterpret_cast<const uint4*>(vb);
    const uint4* seen4 = reinterpret_cast<const uint4*>(seen);
    const int nq = nwp >> 2;
    int total = 0;
    for (int k = 0; k < nv; ++k) {
        // best key (gain << 16 | 0xffff - view) of the lane's candidates
        // (gain < 2^15, views < 2^16), then the wave's on the DPP network
        int key = -1;
        for (int c = lane; c < nv; c += 64) {
            if (taken[c]) continue;
            int cnt = 0;
            for (int q = 0; q < nq; ++q) {
                const uint4 x = vb4[(size_t)c * nq + q], y = seen4[q];
                cnt += __popc(x.x & ~y.x) + __popc(x.y & ~y.y) + __popc(x.z & ~y.z) + __popc(x.w & ~y.w);
            }
            key = max(key, (cnt << 16) | (0xffff - c));
        }
        key = row_max(key);
        key = max(max(__builtin_amdgcn_readlane(key, 0), __builtin_amdgcn_readlane(key, 16)),
                  max(__builtin_amdgcn_readlane(key, 32), __builtin_amdgcn_readlane(key, 48)));
        const int b = 0xffff - (key & 0xffff);
        total += key >> 16;
        if (lane == 0) {
            taken[b] = 1;
            order[off + k] = hand_views[off + b];
            covered[off + k] = total;
        }
        for (int wd = lane; wd < nwp; wd += 64) seen[wd] |= vb[(size_t)b * nwp + wd];
        wave_lds_sync();   // the next step reads seen and taken
    }
}

__global__ void k_fill_i32(int* __restrict__ p, long long n, int v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_u64(unsigned long long* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void k_fill(float* __restrict__ p, long long n, float v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace hr
