// Learned edge-sampling proposal (a project addition to the silhouette
// sampling of Section 4.2.2): per (view, silhouette edge) features, a
// 16-64-64-1 network with erf-GELU evaluated on MFMA (bfloat16 operands,
// float32 accumulation), integer sampling weights and their CDF, per-edge
// statistics of the sampled boundary term, online training of the network by
// the KL divergence from the statistics, and Adam on float32 master weights.
//
// Layout conventions of __builtin_amdgcn_mfma_f32_16x16x16bf16_1k (one wave;
// lane l, r = l % 16, g = l / 16, i = 0..3):
//   A[m][k]: lane holds A[r][4g + i];  B[k][n]: lane holds B[4g + i][r];
//   D[m][n]: lane holds D[4g + i][r].
// The network runs transposed (D^T = W^T X^T), so that a row of the batch
// lives in lane r of every lane group and the layer-1 output registers are the
// layer-2 B operands as they stand.
#pragma once

#include "kernels.h"

namespace hr {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 16, kMlpHid = 64;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHid;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid;
constexpr int kMlpParams = kOffB3 + 1;     // 5313
constexpr int kPropMaxEdges = 8192;
constexpr int kFitMaxRows = 16384;
// fb: float operands of the network (b1, b2, bfloat16 values of w3, b3)
constexpr int kFbB1 = 0, kFbB2 = 64, kFbW3 = 128, kFbB3 = 192, kFbSize = 193;

struct PropDev {
    float* theta;        // [kMlpParams] master parameters
    float* m;            // Adam moments
    float* v;
    float* grad;         // gradient accumulator (cleared by the Adam step)
    int* step;           // Adam step count
    s4v* w1p;            // [4][64]     layer-1 A operands (W1^T tiles)
    s4v* w2p;            // [4][4][64]  layer-2 A operands (W2^T tiles; mt output, kt input)
    s4v* w2bp;           // [4][4][64]  backward A operands (W2 tiles; mt input, kt output)
    float* fb;           // [kFbSize]
    float* z;            // [nV,E] logits of the last proposal pass
    s4v* feat;           // [nV,E,4] the 16 bfloat16 inputs of each row
    float* stat_a;       // [nV,E] sum of |sample contribution|
    float* stat_dc;      // [nV,E,4] sum of |c- - c+| per channel, sample count
    float* ema;          // [nV,E,4] colour-jump averages, [3] = 1 once measured
    const float* z_override;   // nullable [nV,E]: logits used instead of the network
    unsigned short* list;      // [nV,E] silhouette edges of each view (edge order)
    int* nlist;                // [nV]
    double* vstat;             // [nV,2] max logit, sum w exp(z - max) of each view
    int* vcount;               // [nV] finished blocks of the proposal pass (reset by the last)
    int* tcount;               // [1] finished blocks of the training pass (reset by the last)
    float eps, ema_beta, lr, beta1, beta2, adam_eps;
    int split;                 // blocks per view of the proposal and training passes
};

__device__ __forceinline__ unsigned short bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad_f(float x)
{
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

__device__ __forceinline__ f4v mfma16(s4v a, s4v b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

struct MlpRegs {
    s4v w1[4];
    s4v w2[16];
};

__device__ __forceinline__ void load_mlp(const PropDev& P, int lane, MlpRegs& R)
{
#pragma unroll
    for (int t = 0; t < 4; ++t) R.w1[t] = P.w1p[t * 64 + lane];
#pragma unroll
    for (int t = 0; t < 16; ++t) R.w2[t] = P.w2p[t * 64 + lane];
}

// pre-activations and hidden values of one 16-row tile (transposed layout:
// lane (r, g) holds row r, hidden units 16 mt + 4 g + i)
struct TileFwd {
    f4v a1[4];
    s4v h1[4];
    f4v a2[4];
};

// Logit of the lane's row (valid in every lane group).
__device__ __forceinline__ float mlp_tile_fwd(const MlpRegs& R, const float* __restrict__ fb, s4v x, int g,
                                              TileFwd& T)
{
    const f4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f4v c = mfma16(R.w1[mt], x, zero);
        s4v h;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            c[i] += fb[kFbB1 + 16 * mt + 4 * g + i];
            h[i] = (short)bf16_bits(gelu_f(c[i]));
        }
        T.a1[mt] = c;
        T.h1[mt] = h;
    }
    float zp = 0.0f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f4v c = zero;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) c = mfma16(R.w2[mt * 4 + kt], T.h1[kt], c);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            c[i] += fb[kFbB2 + 16 * mt + 4 * g + i];
            zp += bf16_val(bf16_bits(gelu_f(c[i]))) * fb[kFbW3 + 16 * mt + 4 * g + i];
        }
        T.a2[mt] = c;
    }
    zp += __shfl_xor(zp, 16, 64);
    zp += __shfl_xor(zp, 32, 64);
    return zp + fb[kFbB3];
}

__device__ __forceinline__ s4v pack_bf16(const float f[4])
{
    s4v x;
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = (short)bf16_bits(f[i]);
    return x;
}

// Sum of v over the 16 lanes of each row (lane group), complete in the row's
// last lane (r = 15): four DPP row shifts.
__device__ __forceinline__ float row16_sum(float v)
{
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));   // row_shr:1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));   // row_shr:2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));   // row_shr:4
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));   // row_shr:8
    return v;
}

// weight-gradient accumulators of one wave (MFMA accumulators kept across tiles)
struct GradAcc {
    f4v dw2[16];   // tile (mt input, nt output): lane holds dW2[16 mt + 4 g + i][16 nt + r]
    f4v dw1[4];    // tile nt: lane holds dW1[4 g + i][16 nt + r]
};

__device__ __forceinline__ void grad_acc_zero(GradAcc& G)
{
    const f4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int t = 0; t < 16; ++t) G.dw2[t] = zero;
#pragma unroll
    for (int t = 0; t < 4; ++t) G.dw1[t] = zero;
}

// add a wave's weight gradients to `gl` (LDS, kMlpParams floats)
__device__ __forceinline__ void grad_acc_flush(const GradAcc& G, int r, int g, float* gl)
{
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                atomicAdd(gl + kOffW2 + (16 * mt + 4 * g + i) * 64 + 16 * nt + r, G.dw2[mt * 4 + nt][i]);
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) atomicAdd(gl + kOffW1 + (4 * g + i) * 64 + 16 * nt + r, G.dw1[nt][i]);
}

// Back-propagation of dL/dz of the lane's row through one tile.  Bias and
// output-weight gradients are summed over the tile's rows and added to `gl`
// (LDS); the weight-matrix gradients accumulate in G.  tA, tB: this wave's
// LDS transpose buffers (16 x 64 bfloat16 each).
__device__ void mlp_tile_bwd(const s4v* w2b, const float* __restrict__ fb, s4v x, const TileFwd& T, float dz,
                             int r, int g, float* gl, GradAcc& G, unsigned short* tA, unsigned short* tB)
{
    const f4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
    s4v da2b[4];
    const float dzs = row16_sum(dz);
    if (r == 15 && g == 0) atomicAdd(gl + kOffB3, dzs);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int h = 16 * mt + 4 * g + i;
            const float h2 = bf16_val(bf16_bits(gelu_f(T.a2[mt][i])));
            const float da2 = dz * fb[kFbW3 + h] * gelu_grad_f(T.a2[mt][i]);
            const float sw3 = row16_sum(dz * h2), sb2 = row16_sum(da2);
            if (r == 15) {
                atomicAdd(gl + kOffW3 + h, sw3);
                atomicAdd(gl + kOffB2 + h, sb2);
            }
            da2b[mt][i] = (short)bf16_bits(da2);
        }
    }
    // dH1^T = W2 dA2^T; dA1 = dH1 * gelu'(A1)
    s4v da1b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f4v c = zero;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) c = mfma16(w2b[mt * 4 + kt], da2b[kt], c);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int h = 16 * mt + 4 * g + i;
            const float da1 = c[i] * gelu_grad_f(T.a1[mt][i]);
            const float sb1 = row16_sum(da1);
            if (r == 15) atomicAdd(gl + kOffB1 + h, sb1);
            da1b[mt][i] = (short)bf16_bits(da1);
        }
    }
    // dW2 += H1^T dA2 (rows are the contraction): transpose both through LDS
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            tA[r * 64 + 16 * kt + 4 * g + i] = (unsigned short)T.h1[kt][i];
            tB[r * 64 + 16 * kt + 4 * g + i] = (unsigned short)da2b[kt][i];
        }
    wave_lds_sync();
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        s4v A;
#pragma unroll
        for (int i = 0; i < 4; ++i) A[i] = (short)tA[(4 * g + i) * 64 + 16 * mt + r];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            s4v B;
#pragma unroll
            for (int i = 0; i < 4; ++i) B[i] = (short)tB[(4 * g + i) * 64 + 16 * nt + r];
            G.dw2[mt * 4 + nt] = mfma16(A, B, G.dw2[mt * 4 + nt]);
        }
    }
    wave_lds_sync();
    // dW1 += X^T dA1
#pragma unroll
    for (int i = 0; i < 4; ++i) tA[r * 16 + 4 * g + i] = (unsigned short)x[i];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
        for (int i = 0; i < 4; ++i) tB[r * 64 + 16 * kt + 4 * g + i] = (unsigned short)da1b[kt][i];
    wave_lds_sync();
    s4v A;
#pragma unroll
    for (int i = 0; i < 4; ++i) A[i] = (short)tA[(4 * g + i) * 16 + r];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        s4v B;
#pragma unroll
        for (int i = 0; i < 4; ++i) B[i] = (short)tB[(4 * g + i) * 64 + 16 * nt + r];
        G.dw1[nt] = mfma16(A, B, G.dw1[nt]);
    }
    wave_lds_sync();
}

// operand copies of the master parameters (one block)
__device__ void pack_operands(const PropDev& P)
{
    const float* th = P.theta;
    unsigned short* w1p = reinterpret_cast<unsigned short*>(P.w1p);
    unsigned short* w2p = reinterpret_cast<unsigned short*>(P.w2p);
    unsigned short* w2bp = reinterpret_cast<unsigned short*>(P.w2bp);
    for (int idx = threadIdx.x; idx < kMlpIn * kMlpHid; idx += blockDim.x) {
        const int k = idx / kMlpHid, j = idx % kMlpHid;   // W1[k][j]
        const int mt = j / 16, l = 16 * (k / 4) + (j % 16), i = k % 4;
        w1p[(mt * 64 + l) * 4 + i] = bf16_bits(th[kOffW1 + idx]);
    }
    for (int idx = threadIdx.x; idx < kMlpHid * kMlpHid; idx += blockDim.x) {
        const int k = idx / kMlpHid, j = idx % kMlpHid;   // W2[k][j]: input k, output j
        const unsigned short b = bf16_bits(th[kOffW2 + idx]);
        {   // A = W2^T: m = j, kk = k
            const int mt = j / 16, kt = k / 16, l = 16 * ((k % 16) / 4) + (j % 16), i = k % 4;
            w2p[((mt * 4 + kt) * 64 + l) * 4 + i] = b;
        }
        {   // A = W2: m = k, kk = j
            const int mt = k / 16, kt = j / 16, l = 16 * ((j % 16) / 4) + (k % 16), i = j % 4;
            w2bp[((mt * 4 + kt) * 64 + l) * 4 + i] = b;
        }
    }
    for (int idx = threadIdx.x; idx < kMlpHid; idx += blockDim.x) {
        P.fb[kFbB1 + idx] = th[kOffB1 + idx];
        P.fb[kFbB2 + idx] = th[kOffB2 + idx];
        P.fb[kFbW3 + idx] = bf16_val(bf16_bits(th[kOffW3 + idx]));
    }
    if (threadIdx.x == 0) P.fb[kFbB3] = th[kOffB3];
}

__global__ void __launch_bounds__(256) k_proposal_pack(PropDev P) { pack_operands(P); }

// Adam on the master parameters with the accumulated gradient, then the
// operand copies (one block).
__device__ void adam_and_pack(const PropDev& P)
{
    const int t = *P.step + 1;
    __syncthreads();
    if (threadIdx.x == 0) *P.step = t;
    const double bc1 = 1.0 - pow((double)P.beta1, (double)t), bc2 = 1.0 - pow((double)P.beta2, (double)t);
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) {
        const float g = P.grad[i];
        const float m2 = P.beta1 * P.m[i] + (1.0f - P.beta1) * g;
        const float v2 = P.beta2 * P.v[i] + (1.0f - P.beta2) * g * g;
        P.m[i] = m2;
        P.v[i] = v2;
        P.theta[i] -= P.lr * (float)(m2 / bc1) / (sqrtf((float)(v2 / bc2)) + P.adam_eps);
        P.grad[i] = 0.0f;
    }
    __syncthreads();
    pack_operands(P);
}

__global__ void __launch_bounds__(256) k_proposal_adam(PropDev P) { adam_and_pack(P); }

// Silhouette edges of view vi (w > 0) in edge order -> list; returns the count.
__device__ int silhouette_list(const EdgeRec* __restrict__ rec, int E, unsigned short* list, int* part)
{
    const int per = (E + blockDim.x - 1) / blockDim.x;
    const int e0 = threadIdx.x * per, e1 = min(E, e0 + per);
    int n = 0;
    for (int e = e0; e < e1; ++e) n += rec[e].w > 0;
    part[threadIdx.x] = n;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
        const int x = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    int pos = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
    for (int e = e0; e < e1; ++e)
        if (rec[e].w > 0) list[pos++] = (unsigned short)e;
    const int total = part[blockDim.x - 1];
    __syncthreads();
    return total;
}

// Colour-map value at (u, v): texel centres at ((j + 0.5)/T_w, (i + 0.5)/T_h),
// clamp to edge.
__device__ __forceinline__ void tex_bilinear(const float* __restrict__ tex, int th, int tw, float u, float v,
                                             float out[3])
{
    const float x = u * tw - 0.5f, y = v * th - 0.5f;
    const float fx0 = floorf(x), fy0 = floorf(y);
    const float ax = x - fx0, ay = y - fy0;
    int j0 = (int)fx0, i0 = (int)fy0;
    const int j1 = min(max(j0 + 1, 0), tw - 1), i1 = min(max(i0 + 1, 0), th - 1);
    j0 = min(max(j0, 0), tw - 1);
    i0 = min(max(i0, 0), th - 1);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
        out[ch] = (1.0f - ax) * (1.0f - ay) * tex[3 * (i0 * tw + j0) + ch] + ax * (1.0f - ay) * tex[3 * (i0 * tw + j1) + ch]
                  + (1.0f - ax) * ay * tex[3 * (i1 * tw + j0) + ch] + ax * ay * tex[3 * (i1 * tw + j1) + ch];
}

// Features 4g .. 4g+3 of edge e in view vi (zeros for e < 0):
//  0-3 clipped endpoints over (W, H); 4 clipped length over the diagonal;
//  5, 6 larger / smaller of n_f . vhat over the adjacent faces; 7-9 colour
//  jump (running average of measured |c- - c+|, else |shade - background| at
//  the edge midpoint); 10-15 zero.
__device__ void edge_feature4(const EdgeArgs& a, const float* __restrict__ ema, int vi, int e, int g, float f[4])
{
    f[0] = f[1] = f[2] = f[3] = 0.0f;
    if (e < 0 || g == 3) return;
    const ViewDev& c = a.views[vi];
    const EdgeRec r = a.rec[(size_t)vi * a.m.E + e];
    const float dx = r.bx - r.ax, dy = r.by - r.ay;
    const float W = (float)c.W, H = (float)c.H;
    if (g == 0) {
        f[0] = (r.ax + r.t0 * dx) / W;
        f[1] = (r.ay + r.t0 * dy) / H;
        f[2] = (r.ax + r.t1 * dx) / W;
        f[3] = (r.ay + r.t1 * dy) / H;
        return;
    }
    const int va = a.m.edges[2 * e], vb = a.m.edges[2 * e + 1];
    float dc[3];
    const float4 ev = *reinterpret_cast<const float4*>(ema + ((size_t)vi * a.m.E + e) * 4);
    if (ev.w != 0.0f) {
        dc[0] = ev.x; dc[1] = ev.y; dc[2] = ev.z;
    } else {
        const float* nh = a.normals + (size_t)c.hand * a.m.V * 3;
        const float um = 0.5f * (a.uv[2 * va] + a.uv[2 * vb]);
        const float vm = 0.5f * (a.uv[2 * va + 1] + a.uv[2 * vb + 1]);
        float nm[3] = {nh[3 * va] + nh[3 * vb], nh[3 * va + 1] + nh[3 * vb + 1], nh[3 * va + 2] + nh[3 * vb + 2]};
        const float il = 1.0f / sqrtf(nm[0] * nm[0] + nm[1] * nm[1] + nm[2] * nm[2]);
        const float ndl = (nm[0] * a.shading.l[0] + nm[1] * a.shading.l[1] + nm[2] * a.shading.l[2]) * il;
        const float sh = a.shading.ka + a.shading.kd * fmaxf(ndl, 0.0f);
        float col[3];
        tex_bilinear(a.albedo + (size_t)c.hand * a.tex_h * a.tex_w * 3, a.tex_h, a.tex_w, um, vm, col);
        const int px = min(max((int)floorf(0.5f * (r.ax + r.bx)), 0), c.W - 1);
        const int py = min(max((int)floorf(0.5f * (r.ay + r.by)), 0), c.H - 1);
        const float* bg = a.background + 3 * (c.pix0 + (long long)py * c.W + px);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) dc[ch] = fabsf(col[ch] * sh - bg[ch]);
    }
    if (g == 2) {
        f[0] = dc[1];
        f[1] = dc[2];
        return;
    }
    f[0] = sqrtf(dx * dx + dy * dy) * (r.t1 - r.t0) / sqrtf(W * W + H * H);
    const float* vh = a.verts + (size_t)c.hand * a.m.V * 3;
    const float mid[3] = {0.5f * (vh[3 * va] + vh[3 * vb]), 0.5f * (vh[3 * va + 1] + vh[3 * vb + 1]),
                          0.5f * (vh[3 * va + 2] + vh[3 * vb + 2])};
    float vd[3] = {c.o[0] - mid[0], c.o[1] - mid[1], c.o[2] - mid[2]};
    const float iv = 1.0f / sqrtf(vd[0] * vd[0] + vd[1] * vd[1] + vd[2] * vd[2]);
    float dots[2] = {0.0f, 0.0f};
    for (int k = 0; k < 2; ++k) {
        const int fi = a.m.edge_faces[2 * e + k];
        if (fi < 0) continue;
        const float* p0 = vh + 3 * a.m.faces[3 * fi];
        const float* p1 = vh + 3 * a.m.faces[3 * fi + 1];
        const float* p2 = vh + 3 * a.m.faces[3 * fi + 2];
        const float u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        const float w[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        const float n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        const float inn = 1.0f / sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        dots[k] = (n[0] * vd[0] + n[1] * vd[1] + n[2] * vd[2]) * inn * iv;
    }
    f[1] = fmaxf(dots[0], dots[1]);
    f[2] = fminf(dots[0], dots[1]);
    f[3] = dc[0];
}

// Block (v, sp) of grid (n_views, split): features and logits of tiles
// sp, sp + split, ... of view v's silhouette edges.  The last block of a view
// to finish then derives the integer sampling weights
// W_e = max(1, floor(w_e (1 + (1 - eps)(E_e/Ebar - 1)))), E_e = exp(z_e - max z),
// Ebar = sum w E / sum w (equal logits keep the length weights exactly), their
// inclusive prefix sums and total, and keeps (max z, sum w E) for training.
__global__ void __launch_bounds__(256) k_proposal(EdgeArgs a, PropDev P)
{
    __shared__ unsigned short list[kPropMaxEdges];
    __shared__ float zl[kPropMaxEdges];
    __shared__ int ipart[256];
    __shared__ double dpart[256];
    __shared__ unsigned long long upart[256];
    __shared__ int last;
    const int vi = blockIdx.x, sp = blockIdx.y, S = gridDim.y;
    const int E = a.m.E;
    EdgeRec* rec = a.rec + (size_t)vi * E;
    const int n = silhouette_list(rec, E, list, ipart);
    if (sp == 0) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) P.list[(size_t)vi * E + j] = list[j];
        if (threadIdx.x == 0) P.nlist[vi] = n;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    const bool use_net = P.z_override == nullptr;
    MlpRegs R;
    if (use_net) load_mlp(P, lane, R);
    for (int t = 4 * sp + wave; 16 * t < n; t += 4 * S) {
        const int row = 16 * t + r;
        const int e = row < n ? (int)list[row] : -1;
        float f[4];
        edge_feature4(a, P.ema, vi, e, g, f);
        const s4v x = pack_bf16(f);
        if (e >= 0) P.feat[((size_t)vi * E + e) * 4 + g] = x;
        float z;
        if (use_net) {
            TileFwd T;
            z = mlp_tile_fwd(R, P.fb, x, g, T);
        } else {
            z = e >= 0 ? P.z_override[(size_t)vi * E + e] : 0.0f;
        }
        if (e >= 0 && g == 0) P.z[(size_t)vi * E + e] = z;
    }
    // the last block of the view continues
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(P.vcount + vi, 1) == S - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (threadIdx.x == 0) P.vcount[vi] = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) zl[j] = P.z[(size_t)vi * E + list[j]];
    __syncthreads();
    // max logit, then sum w exp(z - max) and sum w
    float zm = -3.0e38f;
    for (int j = threadIdx.x; j < n; j += blockDim.x) zm = fmaxf(zm, zl[j]);
    dpart[threadIdx.x] = zm;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) dpart[threadIdx.x] = fmax(dpart[threadIdx.x], dpart[threadIdx.x + o]);
        __syncthreads();
    }
    const double zmax = dpart[0];
    __syncthreads();
    double s1 = 0.0;
    unsigned long long s0 = 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const uint32_t w = rec[list[j]].w;
        s1 += (double)w * exp((double)zl[j] - zmax);
        s0 += w;
    }
    dpart[threadIdx.x] = s1;
    upart[threadIdx.x] = s0;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            dpart[threadIdx.x] += dpart[threadIdx.x + o];
            upart[threadIdx.x] += upart[threadIdx.x + o];
        }
        __syncthreads();
    }
    const double S1 = dpart[0];
    const double ebar = n > 0 ? S1 / (double)upart[0] : 1.0;
    if (threadIdx.x == 0) {
        P.vstat[2 * vi] = zmax;
        P.vstat[2 * vi + 1] = S1;
    }
    __syncthreads();
    // weights of a contiguous chunk of list entries, block scan, CDF in edge order
    const int per = (n + blockDim.x - 1) / blockDim.x;
    const int j0 = min(n, (int)threadIdx.x * per), j1 = min(n, j0 + per);
    unsigned long long run = 0;
    for (int j = j0; j < j1; ++j) {
        const uint32_t w = rec[list[j]].w;
        const double ratio = 1.0 + (1.0 - (double)P.eps) * (exp((double)zl[j] - zmax) / ebar - 1.0);
        double Wd = floor((double)w * ratio);
        Wd = fmin(fmax(Wd, 1.0), 4294967295.0);
        const uint32_t Wq = (uint32_t)Wd;
        rec[list[j]].wq = Wq;
        run += Wq;
    }
    upart[threadIdx.x] = run;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
        const unsigned long long x = threadIdx.x >= (unsigned)o ? upart[threadIdx.x - o] : 0ull;
        __syncthreads();
        upart[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned long long* cdf = a.cdf + (size_t)vi * E;
    unsigned long long acc = threadIdx.x > 0 ? upart[threadIdx.x - 1] : 0ull;
    if (threadIdx.x == 0) {
        const int first = n > 0 ? (int)list[0] : E;
        for (int e = 0; e < first; ++e) cdf[e] = 0ull;
    }
    for (int j = j0; j < j1; ++j) {
        acc += rec[list[j]].wq;
        const int eb = list[j], ee = j + 1 < n ? (int)list[j + 1] : E;
        for (int e = eb; e < ee; ++e) cdf[e] = acc;
    }
    if (threadIdx.x == blockDim.x - 1) a.total[vi] = upart[blockDim.x - 1];
}

// Gradient of sum over views of KL(pi || q) from the records of the last
// backward pass: pi = a / sum a, q = w exp(z) / sum w exp(z) of each view's
// silhouette edges (dL/dz = q - pi).  Work item k = (view k / split, part
// k % split) covers tiles part, part + split, ... of the view; a block walks
// items blockIdx.x, blockIdx.x + gridDim.x, ... and adds its gradient to
// P.grad once.  The last block to finish takes the Adam step.
__global__ void __launch_bounds__(256) k_proposal_train(const EdgeRec* __restrict__ rec, int E, int n_views,
                                                        PropDev P)
{
    __shared__ unsigned short list[kPropMaxEdges];
    __shared__ float gl[kMlpParams];
    __shared__ unsigned short tA[4][16 * 64], tB[4][16 * 64];
    __shared__ double dpart[256];
    __shared__ int last;
    const int S = P.split;
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) gl[i] = 0.0f;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    MlpRegs R;
    load_mlp(P, lane, R);
    s4v w2b[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) w2b[t] = P.w2bp[t * 64 + lane];
    GradAcc G;
    grad_acc_zero(G);
    bool any = false;
    for (int k = blockIdx.x; k < n_views * S; k += gridDim.x) {
        const int vi = k / S, sp = k % S;
        const int n = P.nlist[vi];
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += blockDim.x) list[j] = P.list[(size_t)vi * E + j];
        const float* zv = P.z + (size_t)vi * E;
        const float* av = P.stat_a + (size_t)vi * E;
        double sa = 0.0;
        for (int j = threadIdx.x; j < n; j += blockDim.x) sa += (double)av[list[j]];
        dpart[threadIdx.x] = sa;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) dpart[threadIdx.x] += dpart[threadIdx.x + o];
            __syncthreads();
        }
        const double Sa = dpart[0];
        if (!(Sa > 0.0) || n == 0) continue;
        any = true;
        const double zmax = P.vstat[2 * vi], S1 = P.vstat[2 * vi + 1];
        for (int t = 4 * sp + wave; 16 * t < n; t += 4 * S) {
            const int row = 16 * t + r;
            const int e = row < n ? (int)list[row] : -1;
            s4v x = {0, 0, 0, 0};
            float dz = 0.0f;
            if (e >= 0) {
                x = P.feat[((size_t)vi * E + e) * 4 + g];
                // the proposal pass recorded the view's normaliser sum w exp(z - max z)
                const double q = (double)rec[(size_t)vi * E + e].w * exp((double)zv[e] - zmax) / S1;
                dz = (float)(q - (double)av[e] / Sa);
            }
            TileFwd T;
            (void)mlp_tile_fwd(R, P.fb, x, g, T);
            mlp_tile_bwd(w2b, P.fb, x, T, dz, r, g, gl, G, tA[wave], tB[wave]);
        }
    }
    grad_acc_flush(G, r, g, gl);
    __syncthreads();
    if (__syncthreads_or(any))
        for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x)
            if (gl[i] != 0.0f) unsafeAtomicAdd(P.grad + i, gl[i]);
    // the last block takes the Adam step
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(P.tcount, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (threadIdx.x == 0) *P.tcount = 0;
    adam_and_pack(P);
}

// Colour-jump averages of the edges sampled since the last call, statistics
// cleared (grid-stride over all (view, edge) rows).
__global__ void __launch_bounds__(256) k_proposal_ema(PropDev P, long long rows)
{
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < rows;
         k += (long long)gridDim.x * blockDim.x) {
        float4 dc = reinterpret_cast<const float4*>(P.stat_dc)[k];
        if (dc.w > 0.0f) {
            float4 em = reinterpret_cast<const float4*>(P.ema)[k];
            const float inv = 1.0f / dc.w;
            const float m0 = dc.x * inv, m1 = dc.y * inv, m2 = dc.z * inv;
            if (em.w != 0.0f) {
                em.x = P.ema_beta * em.x + (1.0f - P.ema_beta) * m0;
                em.y = P.ema_beta * em.y + (1.0f - P.ema_beta) * m1;
                em.z = P.ema_beta * em.z + (1.0f - P.ema_beta) * m2;
            } else {
                em.x = m0; em.y = m1; em.z = m2;
            }
            em.w = 1.0f;
            reinterpret_cast<float4*>(P.ema)[k] = em;
        }
        reinterpret_cast<float4*>(P.stat_dc)[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        P.stat_a[k] = 0.0f;
    }
}

// The network on caller rows X [n,16] (4 tiles of 16 rows per block).
__global__ void __launch_bounds__(256) k_proposal_eval(PropDev P, const float* __restrict__ X, int n,
                                                       float* __restrict__ z)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    const int row = (blockIdx.x * 4 + wave) * 16 + r;
    float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (row < n)
        for (int i = 0; i < 4; ++i) f[i] = X[(size_t)row * 16 + 4 * g + i];
    MlpRegs R;
    load_mlp(P, lane, R);
    TileFwd T;
    const float zz = mlp_tile_fwd(R, P.fb, pack_bf16(f), g, T);
    if (row < n && g == 0) z[row] = zz;
}

// KL gradient of caller rows (one group: a single softmax over the rows with
// w > 0); zs = the rows' logits from k_proposal_eval.  One block.
__global__ void __launch_bounds__(256) k_proposal_fit(PropDev P, const float* __restrict__ X,
                                                      const uint32_t* __restrict__ w, const float* __restrict__ av,
                                                      const float* __restrict__ zs, int n, float* __restrict__ grad_out,
                                                      int apply)
{
    __shared__ float gl[kMlpParams];
    __shared__ unsigned short tA[4][16 * 64], tB[4][16 * 64];
    __shared__ double dpart[256];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) gl[i] = 0.0f;
    float zm = -3.0e38f;
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        if (w[j] > 0) zm = fmaxf(zm, zs[j]);
    dpart[threadIdx.x] = zm;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) dpart[threadIdx.x] = fmax(dpart[threadIdx.x], dpart[threadIdx.x + o]);
        __syncthreads();
    }
    const double zmax = dpart[0];
    __syncthreads();
    double s1 = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        if (w[j] > 0) s1 += (double)w[j] * exp((double)zs[j] - zmax);
    dpart[threadIdx.x] = s1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) dpart[threadIdx.x] += dpart[threadIdx.x + o];
        __syncthreads();
    }
    const double S1 = dpart[0];
    __syncthreads();
    double sa = 0.0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) sa += (double)av[j];
    dpart[threadIdx.x] = sa;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) dpart[threadIdx.x] += dpart[threadIdx.x + o];
        __syncthreads();
    }
    const double Sa = dpart[0];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, g = lane >> 4;
    if (Sa > 0.0) {
        MlpRegs R;
        load_mlp(P, lane, R);
        s4v w2b[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) w2b[t] = P.w2bp[t * 64 + lane];
        GradAcc G;
        grad_acc_zero(G);
        for (int t = wave; 16 * t < n; t += 4) {
            const int row = 16 * t + r;
            float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            float dz = 0.0f;
            if (row < n) {
                for (int i = 0; i < 4; ++i) f[i] = X[(size_t)row * 16 + 4 * g + i];
                const double q = w[row] > 0 ? (double)w[row] * exp((double)zs[row] - zmax) / S1 : 0.0;
                dz = (float)(q - (double)av[row] / Sa);
            }
            const s4v x = pack_bf16(f);
            TileFwd T;
            (void)mlp_tile_fwd(R, P.fb, x, g, T);
            mlp_tile_bwd(w2b, P.fb, x, T, dz, r, g, gl, G, tA[wave], tB[wave]);
        }
        grad_acc_flush(G, r, g, gl);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) {
        if (grad_out) grad_out[i] = gl[i];
        if (apply) P.grad[i] += gl[i];
    }
}

// readback of the stored features (zeros for rows that are not sampled)
__global__ void k_proposal_read_feat(const s4v* __restrict__ feat, const EdgeRec* __restrict__ rec, long long n_rows,
                                     float* __restrict__ out)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_rows * 16;
         i += (long long)gridDim.x * blockDim.x) {
        const long long row = i / 16;
        const int k = (int)(i % 16);
        out[i] = rec[row].w > 0 ? bf16_val((unsigned short)feat[row * 4 + k / 4][k % 4]) : 0.0f;
    }
}

__global__ void k_proposal_read_wq(const EdgeRec* __restrict__ rec, long long n_rows, uint32_t* __restrict__ out)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_rows;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = rec[i].wq;
}

}  // namespace hr
