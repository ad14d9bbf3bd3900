// The paper's full data term (Eq. 3 with f1 = D_c + D_e of Eq. 4): per-camera
// colour transforms r' = T_i R, the L1 colour difference, and the L1
// difference of blurred Canny edge maps B(Canny(.)) (Section 3.1,
// "Rendering" and "Render-and-compare"); the two-level colour map
// V = V_high + V_low nearest-upsampled ("Colour mapping").
//
// Canny: luma 0.299 R + 0.587 G + 0.114 B, 5x5 Gaussian smoothing (sigma 1),
// Sobel / 8, magnitude sqrt(gx^2 + gy^2 + 1e-6), suppression along the
// gradient direction quantised to four orientations, thresholds 0.1 / 0.2 on
// the magnitude, one 8-neighbour hysteresis step; Canny(x) = magnitude at
// the selected pixels.  Every filter reads clamped-to-edge pixels of its own
// input outside the image.  B: 11x11 Gaussian, sigma 5.  All of it in float64
// with the filter taps summed in row-major order; the selection is held fixed
// in the derivative, which flows through the magnitude at selected pixels.
//
// Pixels are processed in the loss chunks (4096 pixels of one view per
// block); every stage is one launch over all views, reading its input's
// neighbours (clamped) from global memory.
#pragma once

#include "kernels.h"

namespace hr {

struct DataTermDev {
    double* w5;          // [25] smoothing weights, row-major
    double* w5s;         // [5] the smoothing's 1-D factor (its transpose runs as a row then a column pass)
    double* w11;         // [121] blur weights
    double* w11s;        // [11] the blur's 1-D factor (the blur runs as a column then a row pass)
    double* grey;        // [P] luma of r' = T R
    double* sm;          // [P] smoothed luma
    double* gx;          // [P]
    double* gy;          // [P]
    double* mag;         // [P]
    uint8_t* flags;      // [P] bit 0 kept by the suppression, bit 1 strong, bit 2 selected
    double* edge;        // [P] Canny: magnitude at selected pixels
    double* blur;        // [P] B(Canny(r'))
    double* g1;          // [P] backward scratch (dE/dgx)
    double* g2;          // [P] backward scratch (dE/dgy)
    double* gb;          // [P] dE/dB(Canny(r')) of the edge term (0 off the mask)
    double* vsum;        // [n_views, 2] sums of |O - r'| and |B(C(O)) - B(C(r'))| over masked pixels
    double* gT;          // [n_views, 9] dE/dT
    float w_e;           // weight of the edge term
    double low, high;    // thresholds
};

// The per-pixel kernels take a 4096-pixel chunk of a view per blockIdx.x
// and split it over gridDim.y = kDtSplit blocks (one pixel per thread at 256
// threads), so a whole image fills the GPU.
#ifndef HR_DT_SPLIT
#define HR_DT_SPLIT 8
#endif
constexpr int kDtSplit = HR_DT_SPLIT;

struct DtArgs {
    const int2* chunks;        // (view, first pixel of the chunk in the view)
    const ViewDev* views;
    const float* image;        // R [P,3]
    const float* T;            // [n_views, 9] (nullable: identity)
    const float* target;       // O [P,3] (loss only)
    const float* target_edges; // B(Canny(O)) [P] (loss only)
    const uint8_t* mask;       // [P] nullable
    const float* view_scale;   // [n_views] 1 / (3 masked pixels) (loss only)
    DataTermDev d;
};

constexpr double kGrey0 = 0.299, kGrey1 = 0.587, kGrey2 = 0.114;
constexpr double kMagEps = 1e-6;

// pixel k of this block's chunk: (view record, in-view index, packed index); false past the view
__device__ __forceinline__ bool dt_pixel(const DtArgs& a, int k, ViewDev& c, int& x, int& y, long long& pg)
{
    const int2 ck = a.chunks[blockIdx.x];
    c = load_view(a.views, ck.x);
    const int pl = ck.y + k;   // a view holds at most 4096 x 4096 pixels
    if (pl >= c.W * c.H) return false;
    y = pl / c.W;
    x = pl - y * c.W;
    pg = c.pix0 + pl;
    return true;
}

__device__ __forceinline__ long long dt_at(const ViewDev& c, int x, int y)
{
    x = min(max(x, 0), c.W - 1);
    y = min(max(y, 0), c.H - 1);
    return c.pix0 + (long long)y * c.W + x;
}

// r'_k = (T_k0 R_0 + T_k1 R_1) + T_k2 R_2 in float64
__device__ __forceinline__ void dt_transform(const DtArgs& a, int view, long long pg, double rp[3])
{
    const double R[3] = {(double)a.image[3 * pg], (double)a.image[3 * pg + 1], (double)a.image[3 * pg + 2]};
    if (!a.T) {
        rp[0] = R[0]; rp[1] = R[1]; rp[2] = R[2];
        return;
    }
    const float* T = a.T + 9 * (size_t)view;
    for (int k = 0; k < 3; ++k)
        rp[k] = ((double)T[3 * k] * R[0] + (double)T[3 * k + 1] * R[1]) + (double)T[3 * k + 2] * R[2];
}

// stage 1: luma of r' = T R
__global__ void __launch_bounds__(256) k_dt_grey(DtArgs a)
{
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        double rp[3];
        dt_transform(a, a.chunks[blockIdx.x].x, pg, rp);
        a.d.grey[pg] = (kGrey0 * rp[0] + kGrey1 * rp[1]) + kGrey2 * rp[2];
    }
}

// stage 2: 5x5 smoothing
__global__ void __launch_bounds__(256) k_dt_smooth(DtArgs a)
{
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        double acc = 0.0;
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j) acc = acc + a.d.w5[5 * i + j] * a.d.grey[dt_at(c, x + j - 2, y + i - 2)];
        a.d.sm[pg] = acc;
    }
}

// stage 3: Sobel gradients and magnitude
__global__ void __launch_bounds__(256) k_dt_grad(DtArgs a)
{
    const double sx[9] = {-0.125, 0.0, 0.125, -0.25, 0.0, 0.25, -0.125, 0.0, 0.125};
    const double sy[9] = {-0.125, -0.25, -0.125, 0.0, 0.0, 0.0, 0.125, 0.25, 0.125};
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        double gx = 0.0, gy = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double v = a.d.sm[dt_at(c, x + j - 1, y + i - 1)];
                gx = gx + sx[3 * i + j] * v;
                gy = gy + sy[3 * i + j] * v;
            }
        a.d.gx[pg] = gx;
        a.d.gy[pg] = gy;
        a.d.mag[pg] = sqrt((gx * gx + gy * gy) + kMagEps);
    }
}

// stage 4: suppression along the quantised gradient direction, thresholds
__global__ void __launch_bounds__(256) k_dt_suppress(DtArgs a)
{
    const double tan1 = sqrt(2.0) - 1.0, tan2 = sqrt(2.0) + 1.0;
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        const double gx = a.d.gx[pg], gy = a.d.gy[pg], M = a.d.mag[pg];
        const double ax = fabs(gx), ay = fabs(gy);
        int dx, dy;   // neighbours (x + dx, y + dy) and (x - dx, y - dy)
        if (ay <= tan1 * ax) { dx = 1; dy = 0; }
        else if (ay >= tan2 * ax) { dx = 0; dy = 1; }
        else if (gx * gy > 0.0) { dx = 1; dy = 1; }
        else { dx = 1; dy = -1; }
        const bool keep = M >= a.d.mag[dt_at(c, x + dx, y + dy)] && M >= a.d.mag[dt_at(c, x - dx, y - dy)];
        const bool strong = keep && M > a.d.high;
        a.d.flags[pg] = (uint8_t)((keep ? 1 : 0) | (strong ? 2 : 0));
    }
}

// stage 5: one hysteresis step and the edge map
__global__ void __launch_bounds__(256) k_dt_hyst(DtArgs a)
{
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        const int f = a.d.flags[pg];
        const double M = a.d.mag[pg];
        bool sel = (f & 2) != 0;
        if (!sel && (f & 1) && M > a.d.low) {
            for (int i = -1; i <= 1 && !sel; ++i)
                for (int j = -1; j <= 1; ++j) {
                    const int xx = x + j, yy = y + i;
                    if ((i || j) && xx >= 0 && yy >= 0 && xx < c.W && yy < c.H &&
                        (a.d.flags[c.pix0 + (long long)yy * c.W + xx] & 2)) { sel = true; break; }
                }
        }
        a.d.edge[pg] = sel ? M : 0.0;
        if (sel) a.d.flags[pg] = (uint8_t)(f | 4);
    }
}

// stage 6: the 11x11 blur, separable: a column pass into `tmp`, then a row
// pass; with the loss: per-view sums of the colour and edge differences and
// dE/dB of the edge term.  With the loss only masked pixels need the blurred
// map (unless it is an output).
__global__ void __launch_bounds__(256) k_dt_blur_col(DtArgs a, double* tmp)
{
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        double acc = 0.0;
        for (int i = 0; i < 11; ++i) acc = acc + a.d.w11s[i] * a.d.edge[dt_at(c, x, y + i - 5)];
        tmp[pg] = acc;
    }
}

template <bool LOSS>
__global__ void __launch_bounds__(256) k_dt_blur(DtArgs a, const double* tmp, float* edge_out)
{
    __shared__ double red[2 * 4];
    const int view = a.chunks[blockIdx.x].x;
    double sc = 0.0, se = 0.0;
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        const bool on = !a.mask || a.mask[pg] != 0;
        double acc = 0.0;
        if (!LOSS || edge_out || on)
            for (int j = 0; j < 11; ++j) acc = acc + a.d.w11s[j] * tmp[dt_at(c, x + j - 5, y)];
        a.d.blur[pg] = acc;
        if (edge_out) edge_out[pg] = (float)acc;
        if (LOSS) {
            double gb = 0.0;
            if (on) {
                double rp[3];
                dt_transform(a, view, pg, rp);
                for (int ch = 0; ch < 3; ++ch) sc += fabs((double)a.target[3 * pg + ch] - rp[ch]);
                const double d = acc - (double)a.target_edges[pg];
                se += fabs(d);
                // dE/dB: w_e sign(B - B_O) / n, with 1 / n = 3 view_scale
                gb = (double)a.d.w_e * (double)((d > 0.0) - (d < 0.0)) * (3.0 * (double)a.view_scale[view]);
            }
            a.d.gb[pg] = gb;
        }
    }
    if (!LOSS) return;
    for (int o = 32; o > 0; o >>= 1) { sc += __shfl_xor(sc, o); se += __shfl_xor(se, o); }
    if ((threadIdx.x & 63) == 0) { red[2 * (threadIdx.x >> 6)] = sc; red[2 * (threadIdx.x >> 6) + 1] = se; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) { sc += red[2 * w]; se += red[2 * w + 1]; }
        atomicAdd(a.d.vsum + 2 * view, sc);
        atomicAdd(a.d.vsum + 2 * view + 1, se);
    }
}

// Taps of a clamped (2r+1)-tap filter along one axis that read pixel q from
// the output position p: the tap offsets t in [lo, hi] with clamp(p + t) = q.
__device__ __forceinline__ bool dt_taps(int p, int q, int r, int n, int& lo, int& hi)
{
    if (n == 1) { lo = -r; hi = r; return true; }
    if (q == 0) { lo = -r; hi = min(r, -p); return lo <= hi; }
    if (q == n - 1) { lo = max(-r, n - 1 - p); hi = r; return lo <= hi; }
    lo = hi = q - p;
    return lo >= -r && lo <= r;
}

// Transposed clamped (2r+1)-tap filter at output pixel (x, y) of a view:
// sum over the input positions p that read (x, y) and their taps of
// w[tap] * g[p].  Far from the border a tap reads (x, y) from p = (x, y) -
// tap only; near it the clamped taps of several positions fold onto it.
template <int R>
__device__ __forceinline__ double dt_adjoint(const ViewDev& c, int x, int y, const double* __restrict__ w,
                                             const double* __restrict__ g)
{
    constexpr int N = 2 * R + 1;
    double acc = 0.0;
    if (x >= R && y >= R && x < c.W - R && y < c.H - R) {
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j)
                acc += w[N * i + j] * g[c.pix0 + (long long)(y - (i - R)) * c.W + (x - (j - R))];
        return acc;
    }
    for (int py = max(0, y - R); py <= min(c.H - 1, y + R); ++py) {
        int ylo, yhi;
        if (!dt_taps(py, y, R, c.H, ylo, yhi)) continue;
        for (int px = max(0, x - R); px <= min(c.W - 1, x + R); ++px) {
            int xlo, xhi;
            if (!dt_taps(px, x, R, c.W, xlo, xhi)) continue;
            double ws = 0.0;
            for (int ty = ylo; ty <= yhi; ++ty)
                for (int tx = xlo; tx <= xhi; ++tx) ws += w[N * (ty + R) + tx + R];
            acc += ws * g[c.pix0 + (long long)py * c.W + px];
        }
    }
    return acc;
}

// transposed clamped (2R+1)-tap filter along one axis (AXIS 0: rows of the
// image, i.e. along x; 1: columns, along y) at output pixel (x, y)
template <int R, int AXIS>
__device__ __forceinline__ double dt_adjoint1(const ViewDev& c, int x, int y, const double* __restrict__ w,
                                              const double* __restrict__ g)
{
    const int q = AXIS == 0 ? x : y, n = AXIS == 0 ? c.W : c.H;
    auto at = [&](int p) { return AXIS == 0 ? c.pix0 + (long long)y * c.W + p : c.pix0 + (long long)p * c.W + x; };
    double acc = 0.0;
    if (q >= R && q < n - R) {
        for (int t = 0; t <= 2 * R; ++t) acc += w[t] * g[at(q - (t - R))];
        return acc;
    }
    for (int p = max(0, q - R); p <= min(n - 1, q + R); ++p) {
        int lo, hi;
        if (!dt_taps(p, q, R, n, lo, hi)) continue;
        double ws = 0.0;
        for (int t = lo; t <= hi; ++t) ws += w[t + R];
        acc += ws * g[at(p)];
    }
    return acc;
}

// backward of the blur's row pass (transposed): into `tmp`
__global__ void __launch_bounds__(256) k_dt_bwd_blur_row(DtArgs a, double* tmp)
{
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        tmp[pg] = dt_adjoint1<5, 0>(c, x, y, a.d.w11s, a.d.gb);
    }
}

// backward 1: through the blur's column pass (transposed, from `tmp`) and the
// magnitude at selected pixels: dE/dgx, dE/dgy
__global__ void __launch_bounds__(256) k_dt_bwd_edge(DtArgs a, const double* tmp)
{
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        const double gc = (a.d.flags[pg] & 4) ? dt_adjoint1<5, 1>(c, x, y, a.d.w11s, tmp) : 0.0;
        const double M = a.d.mag[pg];
        a.d.g1[pg] = gc * a.d.gx[pg] / M;
        a.d.g2[pg] = gc * a.d.gy[pg] / M;
    }
}

// backward 2: through the Sobel filters (transposed, clamped): dE/dsmoothed
__global__ void __launch_bounds__(256) k_dt_bwd_sobel(DtArgs a, double* out)
{
    const double sx[9] = {-0.125, 0.0, 0.125, -0.25, 0.0, 0.25, -0.125, 0.0, 0.125};
    const double sy[9] = {-0.125, -0.25, -0.125, 0.0, 0.0, 0.0, 0.125, 0.25, 0.125};
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        out[pg] = dt_adjoint<1>(c, x, y, sx, a.d.g1) + dt_adjoint<1>(c, x, y, sy, a.d.g2);
    }
}

// backward 3a: the smoothing's row pass, transposed: into `tmp`
__global__ void __launch_bounds__(256) k_dt_bwd_smooth_row(DtArgs a, const double* gs, double* tmp)
{
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        tmp[pg] = dt_adjoint1<2, 0>(c, x, y, a.d.w5s, gs);
    }
}

// backward 3b: through the smoothing's column pass (transposed, from `gs`,
// the row pass's output) and the luma to dE/dr', plus the colour term; then
// dE/dR = T^T dE/dr' and the per-view sums of dE/dT = sum_p dE/dr'_p R_p^T
__global__ void __launch_bounds__(256) k_dt_bwd_final(DtArgs a, const double* gs, float* dimage)
{
    __shared__ double red[9 * 4];
    const int view = a.chunks[blockIdx.x].x;
    double gT[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = blockIdx.y * blockDim.x + threadIdx.x; k < kLossChunk; k += blockDim.x * gridDim.y) {
        ViewDev c; int x, y; long long pg;
        if (!dt_pixel(a, k, c, x, y, pg)) break;
        const double g = dt_adjoint1<2, 1>(c, x, y, a.d.w5s, gs);
        double grp[3] = {kGrey0 * g, kGrey1 * g, kGrey2 * g};
        if (!a.mask || a.mask[pg] != 0) {
            double rp[3];
            dt_transform(a, view, pg, rp);
            const double sc = (double)a.view_scale[view];
            for (int ch = 0; ch < 3; ++ch) {
                const double d = rp[ch] - (double)a.target[3 * pg + ch];
                grp[ch] += (double)((d > 0.0) - (d < 0.0)) * sc;
            }
        }
        const double R[3] = {(double)a.image[3 * pg], (double)a.image[3 * pg + 1], (double)a.image[3 * pg + 2]};
        for (int ch = 0; ch < 3; ++ch) {
            double gr;
            if (a.T) {
                const float* T = a.T + 9 * (size_t)view;
                gr = ((double)T[ch] * grp[0] + (double)T[3 + ch] * grp[1]) + (double)T[6 + ch] * grp[2];
            } else {
                gr = grp[ch];
            }
            dimage[3 * pg + ch] = (float)gr;
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) gT[3 * i + j] += grp[i] * R[j];
    }
    for (int q = 0; q < 9; ++q)
        for (int o = 32; o > 0; o >>= 1) gT[q] += __shfl_xor(gT[q], o);
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 9; ++q) red[9 * (threadIdx.x >> 6) + q] = gT[q];
    __syncthreads();
    if (threadIdx.x < 9) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[9 * w + threadIdx.x];
        atomicAdd(a.d.gT + 9 * view + threadIdx.x, s);
    }
}

// per hand: loss = sum over its views of (colour sum) / (3 n) + w_e (edge sum) / n;
// dE/dT to float (one block)
__global__ void __launch_bounds__(256) k_dt_finish(DtArgs a, const int* hand_view_off, const int* hand_views,
                                                   int n_hands, int n_views, float* loss, float* grad_T)
{
    for (int h = threadIdx.x; h < n_hands; h += blockDim.x) {
        double l = 0.0;
        for (int q = hand_view_off[h]; q < hand_view_off[h + 1]; ++q) {
            const int v = hand_views[q];
            const double s3 = (double)a.view_scale[v];   // 1 / (3 n), 0 for an empty mask
            l += a.d.vsum[2 * v] * s3 + (double)a.d.w_e * a.d.vsum[2 * v + 1] * (3.0 * s3);
        }
        loss[h] = (float)l;
    }
    if (grad_T)
        for (int i = threadIdx.x; i < 9 * n_views; i += blockDim.x) grad_T[i] = (float)a.d.gT[i];
}

__global__ void k_dt_zero(double* p, int n)
{
    for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x) p[i] = 0.0;
}

// V = V_high + V_low nearest-upsampled (th, tw multiples of L)
__global__ void __launch_bounds__(256) k_compose_albedo(const float* __restrict__ low, int L,
                                                        const float* __restrict__ high, float* __restrict__ out,
                                                        int th, int tw, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const long long t = i / 3;
        const int ch = (int)(i - 3 * t);
        const long long h = t / ((long long)th * tw);
        const int r = (int)(t - h * th * tw);
        const int ty = r / tw, tx = r - ty * tw;
        const int ly = ty / (th / L), lx = tx / (tw / L);
        out[i] = high[i] + low[((h * L + ly) * L + lx) * 3 + ch];
    }
}

// dE/dV_low: one block per (hand, low texel), a sum over its block of texels
__global__ void __launch_bounds__(256) k_albedo_low_grad(const float* __restrict__ g, int L, int th, int tw,
                                                         float* __restrict__ out)
{
    __shared__ double red[3 * 4];
    const int cell = blockIdx.x % (L * L), h = blockIdx.x / (L * L);
    const int ly = cell / L, lx = cell - ly * L;
    const int bh = th / L, bw = tw / L;
    double s[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < bh * bw; k += blockDim.x) {
        const int ty = ly * bh + k / bw, tx = lx * bw + k % bw;
        const float* p = g + (((size_t)h * th + ty) * tw + tx) * 3;
        s[0] += p[0]; s[1] += p[1]; s[2] += p[2];
    }
    for (int q = 0; q < 3; ++q)
        for (int o = 32; o > 0; o >>= 1) s[q] += __shfl_xor(s[q], o);
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 3; ++q) red[3 * (threadIdx.x >> 6) + q] = s[q];
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[3 * w + threadIdx.x];
        out[((size_t)h * L * L + cell) * 3 + threadIdx.x] = (float)t;
    }
}

// plain Adam on n values (t >= 1), clamped to [lo, hi]
__global__ void __launch_bounds__(256) k_adam_plain(float* __restrict__ x, const float* __restrict__ g,
                                                    float* __restrict__ m, float* __restrict__ v, long long n,
                                                    float lr, float b1, float b2, float eps, float bc1, float bc2,
                                                    float lo, float hi)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float xi = x[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
        x[i] = fminf(fmaxf(xi, lo), hi);
    }
}

}  // namespace hr

namespace hr {

// loss scale 1 / (3 masked pixels) of every view (one block per view)
__global__ void __launch_bounds__(256) k_dt_scale(const ViewDev* __restrict__ views, const uint8_t* __restrict__ mask,
                                                  float* __restrict__ view_scale)
{
    mask_scale(views, mask, view_scale, blockIdx.x);
}

}  // namespace hr
