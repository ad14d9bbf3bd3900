/*
 * Reference CPU implementation (test infrastructure only: used by tests/, the
 * smoke check and the CPU baseline of the benchmark; never by the product path).
 *
 * A plain, slow, brute-force evaluation of the Monte Carlo render-and-compare
 * estimator of the paper (Section 3.1, Eq. 3 and Eq. 4's colour term; pixels are
 * integrals of samples of the rendering equation, Section 3 "Method"; gradients
 * include visibility edges sampled continuously, Section 4.2.2, following the
 * edge-sampling renderer of Li et al. 2018 that the paper adopts).
 *
 * Precision: all continuous values (ray parameters, barycentrics, shading,
 * gradients) are float64.  Decisions that turn floating point into an integer
 * are taken in float32, exactly as the GPU kernels take them, so that both sides
 * make the same discrete choice:
 *   - which triangle a ray hits first: the watertight ray/triangle test of
 *     Woop, Benthin and Wald (JCGT 2013) evaluated in float32 against every
 *     triangle (no acceleration structure), closest (t, face id) wins;
 *   - which edges are silhouettes, their clipped screen extent and their
 *     quantised sampling weight, the position of every edge sample and of its
 *     two side rays, and the pixel that owns it.
 * Random numbers come from Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 * written here from its published definition.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math: the
 * float32 decision arithmetic must round exactly as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x64-10                                                             */
/* ------------------------------------------------------------------------ */

static void philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* exported for the pin against an independent library implementation */
void ora_philox4x64(const uint64_t* ctr, const uint64_t* key, uint64_t* out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) philox4x64_10(ctr + 4 * i, key, out + 4 * i);
}

/* 24-bit uniforms in [0,1): exact in float32 and float64 */
static float u24_lo(uint64_t r) { return (float)((uint32_t)r >> 8) * 0x1p-24f; }
static float u24_hi(uint64_t r) { return (float)(r >> 40) * 0x1p-24f; }

#define DOMAIN_CAMERA 0ULL
#define DOMAIN_EDGE 1ULL

/* camera sample s of pixel `pix` of global view `view`: screen offsets (u,v) */
static void camera_sample_uv(uint64_t seed, uint32_t iter, int view, int64_t pix, int s,
                             float* u, float* v)
{
    uint64_t ctr[4] = {(uint64_t)pix, (uint64_t)(s >> 2),
                       (uint64_t)(uint32_t)view | (DOMAIN_CAMERA << 32), (uint64_t)iter};
    uint64_t key[2] = {seed, 0};
    uint64_t r[4];
    philox4x64_10(ctr, key, r);
    uint64_t w = r[s & 3];
    *u = u24_lo(w);
    *v = u24_hi(w);
}

/* ------------------------------------------------------------------------ */
/* scene description                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    const float* R;   /* [9] world->camera rotation, row-major */
    const float* o;   /* [3] camera centre */
    float fx, fy, cx, cy;
    int W, H, hand;
    int64_t pix0;     /* first pixel of this view in packed buffers */
} cam_t;

typedef struct {
    int n_verts, n_faces;
    const int32_t* faces;   /* [F,3] */
    const double* uv;       /* [V,2] */
    int tex_h, tex_w;
    double ka, kd, light[3];
} mesh_t;

static cam_t get_cam(const float* R, const float* o, const float* intr, const int32_t* wh,
                     const int32_t* hand, const int64_t* pix_off, int i)
{
    cam_t c;
    c.R = R + 9 * i;
    c.o = o + 3 * i;
    c.fx = intr[4 * i + 0]; c.fy = intr[4 * i + 1];
    c.cx = intr[4 * i + 2]; c.cy = intr[4 * i + 3];
    c.W = wh[2 * i + 0]; c.H = wh[2 * i + 1];
    c.hand = hand[i];
    c.pix0 = pix_off[i];
    return c;
}

/* ------------------------------------------------------------------------ */
/* float32 decisions: ray and watertight ray/triangle test                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    float o[3], d[3];
    int kx, ky, kz;
    float Sx, Sy, Sz;
} ray32_t;

static void ray32_setup(ray32_t* r)
{
    int kz = 0;
    if (fabsf(r->d[1]) > fabsf(r->d[kz])) kz = 1;
    if (fabsf(r->d[2]) > fabsf(r->d[kz])) kz = 2;
    int kx = kz + 1; if (kx == 3) kx = 0;
    int ky = kx + 1; if (ky == 3) ky = 0;
    if (r->d[kz] < 0.0f) { int t = kx; kx = ky; ky = t; }
    r->kx = kx; r->ky = ky; r->kz = kz;
    r->Sx = r->d[kx] / r->d[kz];
    r->Sy = r->d[ky] / r->d[kz];
    r->Sz = 1.0f / r->d[kz];
}

/* ray through screen point (sx,sy): origin = camera centre, direction = R^T dc */
static void ray32_screen(const cam_t* c, float sx, float sy, ray32_t* r)
{
    float dcx = (sx - c->cx) / c->fx;
    float dcy = (sy - c->cy) / c->fy;
    for (int k = 0; k < 3; ++k) {
        float a = c->R[k] * dcx;
        float b = c->R[3 + k] * dcy;
        r->d[k] = (a + b) + c->R[6 + k];
        r->o[k] = c->o[k];
    }
    ray32_setup(r);
}

/* Watertight test.  Returns 1 and t if the ray hits with t > 0. */
static int watertight32(const ray32_t* r, const float v0[3], const float v1[3], const float v2[3],
                        float* t_out)
{
    float A[3], B[3], C[3];
    for (int k = 0; k < 3; ++k) {
        A[k] = v0[k] - r->o[k];
        B[k] = v1[k] - r->o[k];
        C[k] = v2[k] - r->o[k];
    }
    const int kx = r->kx, ky = r->ky, kz = r->kz;
    float Ax = A[kx] - r->Sx * A[kz];
    float Ay = A[ky] - r->Sy * A[kz];
    float Bx = B[kx] - r->Sx * B[kz];
    float By = B[ky] - r->Sy * B[kz];
    float Cx = C[kx] - r->Sx * C[kz];
    float Cy = C[ky] - r->Sy * C[kz];
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
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;
    float det = (U + V) + W;
    if (det == 0.0f) return 0;
    float Az = r->Sz * A[kz];
    float Bz = r->Sz * B[kz];
    float Cz = r->Sz * C[kz];
    float T = (U * Az + V * Bz) + W * Cz;
    float t = T / det;
    if (!(t > 0.0f)) return 0;
    *t_out = t;
    return 1;
}

/* closest hit over all faces: smallest t, ties to the smaller face id; -1 = miss */
static int closest_hit32(const ray32_t* r, const float* v32, const int32_t* faces, int F)
{
    int best = -1;
    float tb = INFINITY;
    for (int f = 0; f < F; ++f) {
        const int32_t* tri = faces + 3 * f;
        float t;
        if (watertight32(r, v32 + 3 * tri[0], v32 + 3 * tri[1], v32 + 3 * tri[2], &t)) {
            if (t < tb) { tb = t; best = f; }
        }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* float64 intersection values and shading                                   */
/* ------------------------------------------------------------------------ */

static void ray64_screen(const cam_t* c, double sx, double sy, double o[3], double d[3])
{
    double dcx = (sx - (double)c->cx) / (double)c->fx;
    double dcy = (sy - (double)c->cy) / (double)c->fy;
    for (int k = 0; k < 3; ++k) {
        d[k] = (double)c->R[k] * dcx + (double)c->R[3 + k] * dcy + (double)c->R[6 + k];
        o[k] = (double)c->o[k];
    }
}

static void sub3(const double* a, const double* b, double* r) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* r)
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

/* barycentrics (b1,b2) and t of the ray's intersection with the plane of the
   triangle, solving o + t d = (1-b1-b2) v0 + b1 v1 + b2 v2 by Cramer's rule */
static void plane_hit64(const double* o, const double* d, const double* v0, const double* v1,
                        const double* v2, double* b1, double* b2, double* t)
{
    double e1[3], e2[3], s[3], p[3], q[3];
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    cross3(d, e2, p);
    double det = dot3(e1, p);
    sub3(o, v0, s);
    cross3(s, e1, q);
    *b1 = dot3(s, p) / det;
    *b2 = dot3(d, q) / det;
    *t = dot3(e2, q) / det;
}

typedef struct {
    int i0, i1, i2;
    double b0, b1, b2;
} hit_t;

/* bilinear albedo lookup with texel centres at (j+1/2)/W, clamp to edge.
   Returns the colour, the four texel indices and weights, and the derivative
   of the colour with respect to the texture coordinates. */
typedef struct {
    int idx[4];
    double w[4];
    double col[3];
    double dcol_du[3], dcol_dv[3];
} texlook_t;

static void tex_lookup(const double* tex, int th, int tw, double u, double v, texlook_t* L)
{
    double x = u * tw - 0.5, y = v * th - 0.5;
    double fx0 = floor(x), fy0 = floor(y);
    double ax = x - fx0, ay = y - fy0;
    int j0 = (int)fx0, i0 = (int)fy0;
    int j1 = j0 + 1, i1 = i0 + 1;
    if (j0 < 0) j0 = 0;
    if (j0 > tw - 1) j0 = tw - 1;
    if (j1 < 0) j1 = 0;
    if (j1 > tw - 1) j1 = tw - 1;
    if (i0 < 0) i0 = 0;
    if (i0 > th - 1) i0 = th - 1;
    if (i1 < 0) i1 = 0;
    if (i1 > th - 1) i1 = th - 1;
    L->idx[0] = i0 * tw + j0; L->w[0] = (1 - ax) * (1 - ay);
    L->idx[1] = i0 * tw + j1; L->w[1] = ax * (1 - ay);
    L->idx[2] = i1 * tw + j0; L->w[2] = (1 - ax) * ay;
    L->idx[3] = i1 * tw + j1; L->w[3] = ax * ay;
    for (int ch = 0; ch < 3; ++ch) {
        double a00 = tex[3 * L->idx[0] + ch], a01 = tex[3 * L->idx[1] + ch];
        double a10 = tex[3 * L->idx[2] + ch], a11 = tex[3 * L->idx[3] + ch];
        L->col[ch] = L->w[0] * a00 + L->w[1] * a01 + L->w[2] * a10 + L->w[3] * a11;
        L->dcol_du[ch] = tw * ((1 - ay) * (a01 - a00) + ay * (a11 - a10));
        L->dcol_dv[ch] = th * ((1 - ax) * (a10 - a00) + ax * (a11 - a01));
    }
}

/* Lambertian + ambient colour of a surface point with interpolated normal */
typedef struct {
    double uv[2];
    double nraw[3], nlen, n[3];
    double ndotl, shade;
    texlook_t tl;
    double col[3];
} shade_t;

static void shade_point(const mesh_t* m, const double* nrm, const double* tex, const hit_t* h,
                        shade_t* S)
{
    const double* uv0 = m->uv + 2 * h->i0;
    const double* uv1 = m->uv + 2 * h->i1;
    const double* uv2 = m->uv + 2 * h->i2;
    S->uv[0] = h->b0 * uv0[0] + h->b1 * uv1[0] + h->b2 * uv2[0];
    S->uv[1] = h->b0 * uv0[1] + h->b1 * uv1[1] + h->b2 * uv2[1];
    const double* n0 = nrm + 3 * h->i0;
    const double* n1 = nrm + 3 * h->i1;
    const double* n2 = nrm + 3 * h->i2;
    for (int k = 0; k < 3; ++k) S->nraw[k] = h->b0 * n0[k] + h->b1 * n1[k] + h->b2 * n2[k];
    S->nlen = sqrt(dot3(S->nraw, S->nraw));
    for (int k = 0; k < 3; ++k) S->n[k] = S->nraw[k] / S->nlen;
    S->ndotl = dot3(S->n, m->light);
    S->shade = m->ka + m->kd * (S->ndotl > 0 ? S->ndotl : 0.0);
    tex_lookup(tex, m->tex_h, m->tex_w, S->uv[0], S->uv[1], &S->tl);
    for (int ch = 0; ch < 3; ++ch) S->col[ch] = S->tl.col[ch] * S->shade;
}

/* Trace the ray through screen point (X,Y) of camera c.  The float32 point
   (sx,sy) (the float32 rounding of (X,Y)) decides the face hit; the float64
   point (X,Y) gives the barycentrics.  Returns the face (or -1). */
static int trace_point(const cam_t* c, const mesh_t* m, const float* v32, const double* v64,
                       float sx, float sy, double X, double Y, hit_t* h)
{
    ray32_t r;
    ray32_screen(c, sx, sy, &r);
    int f = closest_hit32(&r, v32, m->faces, m->n_faces);
    if (f < 0) return -1;
    double o[3], d[3];
    ray64_screen(c, X, Y, o, d);
    const int32_t* tri = m->faces + 3 * f;
    double b1, b2, t;
    plane_hit64(o, d, v64 + 3 * tri[0], v64 + 3 * tri[1], v64 + 3 * tri[2], &b1, &b2, &t);
    h->i0 = tri[0]; h->i1 = tri[1]; h->i2 = tri[2];
    h->b0 = 1.0 - b1 - b2; h->b1 = b1; h->b2 = b2;
    return f;
}

static float* round_verts(const double* v, int n)
{
    float* r = (float*)malloc(sizeof(float) * 3 * (size_t)n);
    for (int i = 0; i < 3 * n; ++i) r[i] = (float)v[i];
    return r;
}

/* ------------------------------------------------------------------------ */
/* forward render                                                            */
/* ------------------------------------------------------------------------ */

/*
 * ora_render: I_p = (1/S) sum_s c(x_{p,s}); c = albedo(uv)*(ka + kd max(0,n.l)) at
 * the first hit, the pixel's background colour on a miss.
 *   verts   [n_hands,V,3] f64     normals [n_hands,V,3] f64 (unit vertex normals)
 *   faces   [F,3] i32             uv [V,2] f64
 *   albedo  [n_hands,th,tw,3] f64 background [P,3] f64 (packed views)
 *   cams: R [n_views,9] f32, o [n_views,3] f32, intr [n_views,4] f32 (fx,fy,cx,cy),
 *         wh [n_views,2] i32, hand [n_views] i32, pix_off [n_views+1] i64
 *   image   [P,3] f64 out;  hit_face [P,spp] i32 out (nullable)
 */
void ora_render(int n_hands, int V, int F, const double* verts, const double* normals,
                const int32_t* faces, const double* uv, int th, int tw, const double* albedo,
                const double* background, int n_views, const float* R, const float* o,
                const float* intr, const int32_t* wh, const int32_t* hand, const int64_t* pix_off,
                const double* shading /* ka, kd, lx, ly, lz */, int spp, uint64_t seed,
                uint32_t iter, double* image, int32_t* hit_face)
{
    mesh_t m = {V, F, faces, uv, th, tw, shading[0], shading[1], {shading[2], shading[3], shading[4]}};
    float* v32 = round_verts(verts, n_hands * V);
    for (int vi = 0; vi < n_views; ++vi) {
        cam_t c = get_cam(R, o, intr, wh, hand, pix_off, vi);
        const float* hv32 = v32 + (size_t)3 * V * c.hand;
        const double* hv64 = verts + (size_t)3 * V * c.hand;
        const double* hn = normals + (size_t)3 * V * c.hand;
        const double* tex = albedo + (size_t)3 * th * tw * c.hand;
        int64_t npix = (int64_t)c.W * c.H;
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            int px = (int)(p % c.W), py = (int)(p / c.W);
            const double* bg = background + 3 * (c.pix0 + p);
            double acc[3] = {0, 0, 0};
            for (int s = 0; s < spp; ++s) {
                float u, v;
                camera_sample_uv(seed, iter, vi, p, s, &u, &v);
                float sx = (float)px + u, sy = (float)py + v;
                hit_t h;
                int f = trace_point(&c, &m, hv32, hv64, sx, sy, px + (double)u, py + (double)v, &h);
                if (hit_face) hit_face[(c.pix0 + p) * spp + s] = f;
                if (f < 0) {
                    for (int ch = 0; ch < 3; ++ch) acc[ch] += bg[ch];
                } else {
                    shade_t S;
                    shade_point(&m, hn, tex, &h, &S);
                    for (int ch = 0; ch < 3; ++ch) acc[ch] += S.col[ch];
                }
            }
            for (int ch = 0; ch < 3; ++ch) image[3 * (c.pix0 + p) + ch] = acc[ch] / spp;
        }
    }
    free(v32);
}

/* ------------------------------------------------------------------------ */
/* interior adjoint (derivative of the estimate at fixed samples)             */
/* ------------------------------------------------------------------------ */

/* Gradient of sum_ch g[ch]*c[ch] for one hit sample.  Accumulates into the
   albedo gradient, the vertex-position gradient (through the hit point, which
   moves with the triangle for a fixed ray) and the vertex-normal gradient. */
static void sample_adjoint(const mesh_t* m, const double* v64, const double* nrm, const double* tex,
                           const double* o, const double* d, const hit_t* h, const double g[3],
                           double* g_tex, double* g_v, double* g_n)
{
    shade_t S;
    shade_point(m, nrm, tex, h, &S);
    /* albedo texels */
    for (int k = 0; k < 4; ++k)
        for (int ch = 0; ch < 3; ++ch) {
            double val = g[ch] * S.shade * S.tl.w[k];
#pragma omp atomic
            g_tex[3 * S.tl.idx[k] + ch] += val;
        }
    double gs = g[0] * S.tl.col[0] + g[1] * S.tl.col[1] + g[2] * S.tl.col[2];
    /* through texture coordinates */
    double g_tu = 0, g_tv = 0;
    for (int ch = 0; ch < 3; ++ch) {
        g_tu += g[ch] * S.shade * S.tl.dcol_du[ch];
        g_tv += g[ch] * S.shade * S.tl.dcol_dv[ch];
    }
    const double* uv0 = m->uv + 2 * h->i0;
    const double* uv1 = m->uv + 2 * h->i1;
    const double* uv2 = m->uv + 2 * h->i2;
    double gb1 = g_tu * (uv1[0] - uv0[0]) + g_tv * (uv1[1] - uv0[1]);
    double gb2 = g_tu * (uv2[0] - uv0[0]) + g_tv * (uv2[1] - uv0[1]);
    /* through the interpolated normal */
    if (S.ndotl > 0) {
        double gn[3], gnr[3];
        for (int k = 0; k < 3; ++k) gn[k] = gs * m->kd * m->light[k];
        double gnn = dot3(gn, S.n);
        for (int k = 0; k < 3; ++k) gnr[k] = (gn[k] - gnn * S.n[k]) / S.nlen;
        const double* n0 = nrm + 3 * h->i0;
        const double* n1 = nrm + 3 * h->i1;
        const double* n2 = nrm + 3 * h->i2;
        for (int k = 0; k < 3; ++k) {
            g_n[3 * h->i0 + k] += h->b0 * gnr[k];
            g_n[3 * h->i1 + k] += h->b1 * gnr[k];
            g_n[3 * h->i2 + k] += h->b2 * gnr[k];
            gb1 += gnr[k] * (n1[k] - n0[k]);
            gb2 += gnr[k] * (n2[k] - n0[k]);
        }
    }
    /* hit point: M [b1,b2,t]^T = o - v0 with M = [v1-v0, v2-v0, -d];
       d[b1,b2,t]/dv_k = -b_k M^{-1}  =>  dE/dv_k = -b_k M^{-T} [gb1, gb2, 0] */
    const double* v0 = v64 + 3 * h->i0;
    const double* v1 = v64 + 3 * h->i1;
    const double* v2 = v64 + 3 * h->i2;
    double Mt[3][3];
    for (int k = 0; k < 3; ++k) {
        Mt[0][k] = v1[k] - v0[k];
        Mt[1][k] = v2[k] - v0[k];
        Mt[2][k] = -d[k];
    }
    /* solve Mt y = rhs where Mt = M^T (rows are the columns of M) */
    double rhs[3] = {gb1, gb2, 0.0};
    double det = Mt[0][0] * (Mt[1][1] * Mt[2][2] - Mt[1][2] * Mt[2][1])
               - Mt[0][1] * (Mt[1][0] * Mt[2][2] - Mt[1][2] * Mt[2][0])
               + Mt[0][2] * (Mt[1][0] * Mt[2][1] - Mt[1][1] * Mt[2][0]);
    double y[3];
    for (int c = 0; c < 3; ++c) {
        double Mc[3][3];
        memcpy(Mc, Mt, sizeof(Mc));
        for (int r = 0; r < 3; ++r) Mc[r][c] = rhs[r];
        double dc = Mc[0][0] * (Mc[1][1] * Mc[2][2] - Mc[1][2] * Mc[2][1])
                  - Mc[0][1] * (Mc[1][0] * Mc[2][2] - Mc[1][2] * Mc[2][0])
                  + Mc[0][2] * (Mc[1][0] * Mc[2][1] - Mc[1][1] * Mc[2][0]);
        y[c] = dc / det;
    }
    (void)o;
    for (int k = 0; k < 3; ++k) {
        g_v[3 * h->i0 + k] -= h->b0 * y[k];
        g_v[3 * h->i1 + k] -= h->b1 * y[k];
        g_v[3 * h->i2 + k] -= h->b2 * y[k];
    }
}

/*
 * ora_backward_interior: gradient of sum_p dimage[p] . I_p with the samples held
 * fixed (the forward's samples are re-drawn from the same counters).
 *   dimage [P,3] f64 (dE/dI)
 *   g_albedo [n_hands,th,tw,3], g_verts [n_hands,V,3], g_normals [n_hands,V,3]:
 *   f64, accumulated into (caller zeroes them).
 */
void ora_backward_interior(int n_hands, int V, int F, const double* verts, const double* normals,
                           const int32_t* faces, const double* uv, int th, int tw,
                           const double* albedo, int n_views, const float* R, const float* o,
                           const float* intr, const int32_t* wh, const int32_t* hand,
                           const int64_t* pix_off, const double* shading, int spp, uint64_t seed,
                           uint32_t iter, const double* dimage, double* g_albedo, double* g_verts,
                           double* g_normals)
{
    mesh_t m = {V, F, faces, uv, th, tw, shading[0], shading[1], {shading[2], shading[3], shading[4]}};
    float* v32 = round_verts(verts, n_hands * V);
    for (int vi = 0; vi < n_views; ++vi) {
        cam_t c = get_cam(R, o, intr, wh, hand, pix_off, vi);
        const float* hv32 = v32 + (size_t)3 * V * c.hand;
        const double* hv64 = verts + (size_t)3 * V * c.hand;
        const double* hn = normals + (size_t)3 * V * c.hand;
        const double* tex = albedo + (size_t)3 * th * tw * c.hand;
        double* gt = g_albedo + (size_t)3 * th * tw * c.hand;
        int64_t npix = (int64_t)c.W * c.H;
        int nthr = 1;
#ifdef _OPENMP
        nthr = omp_get_max_threads();
#endif
        double* gv_t = (double*)calloc((size_t)nthr * 3 * V, sizeof(double));
        double* gn_t = (double*)calloc((size_t)nthr * 3 * V, sizeof(double));
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double* gv = gv_t + (size_t)tid * 3 * V;
            double* gn = gn_t + (size_t)tid * 3 * V;
#pragma omp for schedule(dynamic, 16)
            for (int64_t p = 0; p < npix; ++p) {
                const double* gp = dimage + 3 * (c.pix0 + p);
                if (gp[0] == 0.0 && gp[1] == 0.0 && gp[2] == 0.0) continue;
                double g[3] = {gp[0] / spp, gp[1] / spp, gp[2] / spp};
                int px = (int)(p % c.W), py = (int)(p / c.W);
                for (int s = 0; s < spp; ++s) {
                    float u, v;
                    camera_sample_uv(seed, iter, vi, p, s, &u, &v);
                    float sx = (float)px + u, sy = (float)py + v;
                    double X = px + (double)u, Y = py + (double)v;
                    hit_t h;
                    int f = trace_point(&c, &m, hv32, hv64, sx, sy, X, Y, &h);
                    if (f < 0) continue;
                    double ro[3], rd[3];
                    ray64_screen(&c, X, Y, ro, rd);
                    sample_adjoint(&m, hv64, hn, tex, ro, rd, &h, g, gt, gv, gn);
                }
            }
        }
        double* gvh = g_verts + (size_t)3 * V * c.hand;
        double* gnh = g_normals + (size_t)3 * V * c.hand;
        for (int t = 0; t < nthr; ++t)
            for (int i = 0; i < 3 * V; ++i) {
                gvh[i] += gv_t[(size_t)t * 3 * V + i];
                gnh[i] += gn_t[(size_t)t * 3 * V + i];
            }
        free(gv_t);
        free(gn_t);
    }
    free(v32);
}

/* ------------------------------------------------------------------------ */
/* silhouette edges and edge sampling                                        */
/* ------------------------------------------------------------------------ */

/* float32 projection; returns 0 if the point is not in front of the camera */
static int project32(const cam_t* c, const float* v, float znear, float* px, float* py)
{
    float q0 = v[0] - c->o[0], q1 = v[1] - c->o[1], q2 = v[2] - c->o[2];
    float xc = (c->R[0] * q0 + c->R[1] * q1) + c->R[2] * q2;
    float yc = (c->R[3] * q0 + c->R[4] * q1) + c->R[5] * q2;
    float zc = (c->R[6] * q0 + c->R[7] * q1) + c->R[8] * q2;
    if (!(zc > znear)) return 0;
    *px = (c->fx * xc) / zc + c->cx;
    *py = (c->fy * yc) / zc + c->cy;
    return 1;
}

/* float64 projection and its Jacobian d(px,py)/d(vertex) */
static void project64(const cam_t* c, const double* v, double* pxy, double J[2][3])
{
    double q[3] = {v[0] - c->o[0], v[1] - c->o[1], v[2] - c->o[2]};
    double xc[3];
    for (int r = 0; r < 3; ++r)
        xc[r] = (double)c->R[3 * r] * q[0] + (double)c->R[3 * r + 1] * q[1] + (double)c->R[3 * r + 2] * q[2];
    double z = xc[2];
    pxy[0] = c->fx * xc[0] / z + c->cx;
    pxy[1] = c->fy * xc[1] / z + c->cy;
    double dp[2][3] = {{c->fx / z, 0.0, -c->fx * xc[0] / (z * z)},
                       {0.0, c->fy / z, -c->fy * xc[1] / (z * z)}};
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k)
            J[a][k] = dp[a][0] * c->R[k] + dp[a][1] * c->R[3 + k] + dp[a][2] * c->R[6 + k];
}

/* Liang-Barsky clip of a + t (b-a), t in [0,1], to [0,W]x[0,H] (float32).
   Returns 0 if nothing of positive length remains. */
static int clip32(float ax, float ay, float bx, float by, float W, float H, float* t0, float* t1)
{
    float dx = bx - ax, dy = by - ay;
    float lo = 0.0f, hi = 1.0f;
    float p[4] = {-dx, dx, -dy, dy};
    float q[4] = {ax, W - ax, ay, H - ay};
    for (int k = 0; k < 4; ++k) {
        if (p[k] == 0.0f) {
            if (q[k] < 0.0f) return 0;
        } else {
            float r = q[k] / p[k];
            if (p[k] < 0.0f) { if (r > lo) lo = r; }
            else { if (r < hi) hi = r; }
        }
    }
    if (!(lo < hi)) return 0;
    *t0 = lo; *t1 = hi;
    return 1;
}

typedef struct {
    uint32_t w;          /* quantised weight, 1/256 px units (0 = not sampled) */
    float ax, ay, bx, by; /* projected endpoints */
    float t0, t1;        /* clipped parameter interval */
} edge32_t;

/* Per-view silhouette classification and quantised length weights (float32).
   An edge is a silhouette if it lies on the mesh boundary or its two faces
   face opposite ways as seen from the camera centre. */
static void view_edges(const cam_t* c, const float* v32, const int32_t* faces, int E,
                       const int32_t* edges, const int32_t* edge_faces, edge32_t* out)
{
    const float znear = 1e-4f;
    for (int e = 0; e < E; ++e) {
        edge32_t* r = out + e;
        memset(r, 0, sizeof(*r));
        int a = edges[2 * e], b = edges[2 * e + 1];
        const float* va = v32 + 3 * a;
        int front[2] = {0, 0};
        int nf = edge_faces[2 * e + 1] < 0 ? 1 : 2;
        for (int k = 0; k < nf; ++k) {
            const int32_t* tri = faces + 3 * edge_faces[2 * e + k];
            const float* p0 = v32 + 3 * tri[0];
            const float* p1 = v32 + 3 * tri[1];
            const float* p2 = v32 + 3 * tri[2];
            float e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
            float e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
            float n0 = e1[1] * e2[2] - e1[2] * e2[1];
            float n1 = e1[2] * e2[0] - e1[0] * e2[2];
            float n2 = e1[0] * e2[1] - e1[1] * e2[0];
            float w0 = c->o[0] - va[0], w1 = c->o[1] - va[1], w2 = c->o[2] - va[2];
            float dd = (n0 * w0 + n1 * w1) + n2 * w2;
            front[k] = dd > 0.0f;
        }
        int sil = (nf == 1) || (front[0] != front[1]);
        if (!sil) continue;
        float ax, ay, bx, by;
        if (!project32(c, va, znear, &ax, &ay)) continue;
        if (!project32(c, v32 + 3 * b, znear, &bx, &by)) continue;
        float t0, t1;
        if (!clip32(ax, ay, bx, by, (float)c->W, (float)c->H, &t0, &t1)) continue;
        float dx = bx - ax, dy = by - ay;
        float len = sqrtf(dx * dx + dy * dy);
        if (!(len > 0.0f)) continue;   /* projects to a point: no boundary */
        float ell = len * (t1 - t0);
        float q = floorf(ell * 256.0f);
        uint32_t w = q >= 4294967295.0f ? 0xFFFFFFFFu : (uint32_t)q;
        if (w == 0) w = 1;
        r->w = w;
        r->ax = ax; r->ay = ay; r->bx = bx; r->by = by;
        r->t0 = t0; r->t1 = t1;
    }
}

/*
 * ora_edge_weights: per (view, edge) quantised weights and inclusive prefix sums.
 *   w [n_views,E] u32 out, cdf [n_views,E] u64 out, total [n_views] u64 out,
 *   budget [n_views] i64 out = ceil(total / 256)  (one sample per silhouette pixel),
 *   rec [n_views,E,6] f32 out (nullable): projected endpoints ax, ay, bx, by and
 *   the clipped parameter interval t0, t1 (zeros where w = 0).
 */
void ora_edge_weights(int n_hands, int V, int F, const double* verts, const int32_t* faces, int E,
                      const int32_t* edges, const int32_t* edge_faces, int n_views, const float* R,
                      const float* o, const float* intr, const int32_t* wh, const int32_t* hand,
                      const int64_t* pix_off, uint32_t* w, uint64_t* cdf, uint64_t* total,
                      int64_t* budget, float* rec)
{
    float* v32 = round_verts(verts, n_hands * V);
    edge32_t* ed = (edge32_t*)malloc(sizeof(edge32_t) * (size_t)E);
    for (int vi = 0; vi < n_views; ++vi) {
        cam_t c = get_cam(R, o, intr, wh, hand, pix_off, vi);
        view_edges(&c, v32 + (size_t)3 * V * c.hand, faces, E, edges, edge_faces, ed);
        uint64_t acc = 0;
        for (int e = 0; e < E; ++e) {
            acc += ed[e].w;
            w[(size_t)vi * E + e] = ed[e].w;
            cdf[(size_t)vi * E + e] = acc;
            if (rec) {
                float* r = rec + ((size_t)vi * E + e) * 6;
                r[0] = ed[e].ax; r[1] = ed[e].ay; r[2] = ed[e].bx; r[3] = ed[e].by;
                r[4] = ed[e].t0; r[5] = ed[e].t1;
            }
        }
        total[vi] = acc;
        budget[vi] = (int64_t)((acc + 255) / 256);
    }
    free(ed);
    free(v32);
    (void)F;
}

/*
 * ora_backward_edges: boundary term of the gradient of sum_p dimage[p] . I_p.
 * For each view, `budget` M samples are drawn along silhouette edges: the
 * quantised length weights form an integer CDF of total T; sample k takes a
 * uniform target in the k-th of M strata [k T/M, (k+1) T/M) of it (stratified
 * sampling), picks the edge whose CDF interval holds the target, and a
 * uniform point along the chosen edge.  With stratum width n_k and density
 * (w_e/T)/len_e per unit length, a sample at x on an edge with screen normal n
 * contributes g_p . (c(x - delta n) - c(x + delta n)) * len_e * n_k / w_e
 * times the normal velocity of the edge, split linearly between its endpoints
 * (an unbiased estimate of the boundary integral).
 *   g_verts [n_hands,V,3] f64 accumulated into.
 *   budget_override [n_views] i64 (nullable): number of samples per view.
 *   edge_stats [n_views,E] f64 (nullable): accumulates |g.(c- - c+)| / (pdf M)
 *   per edge (an estimate of each edge's share of the boundary integral).
 *   wq [n_views,E] u32 (nullable): sampling weights replacing the length
 *   weights w_e on silhouette edges (w_e > 0; entries elsewhere are ignored;
 *   each used entry must be >= 1).  The sample budget still follows the
 *   length weights.  Any positive weights give an unbiased estimate.
 *   dc_stats [n_views,E,4] f64 (nullable): accumulates, over the samples whose
 *   pixel has a non-zero dimage, |c- - c+| per channel and the sample count.
 */
void ora_backward_edges(int n_hands, int V, int F, const double* verts, const double* normals,
                        const int32_t* faces, const double* uv, int th, int tw, const double* albedo,
                        const double* background, int E, const int32_t* edges,
                        const int32_t* edge_faces, int n_views, const float* R, const float* o,
                        const float* intr, const int32_t* wh, const int32_t* hand,
                        const int64_t* pix_off, const double* shading, float delta, uint64_t seed,
                        uint32_t iter, const double* dimage, const int64_t* budget_override,
                        double* g_verts, double* edge_stats, const uint32_t* wq, double* dc_stats)
{
    mesh_t m = {V, F, faces, uv, th, tw, shading[0], shading[1], {shading[2], shading[3], shading[4]}};
    float* v32 = round_verts(verts, n_hands * V);
    edge32_t* ed = (edge32_t*)malloc(sizeof(edge32_t) * (size_t)E);
    uint64_t* cdf = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)E);
    for (int vi = 0; vi < n_views; ++vi) {
        cam_t c = get_cam(R, o, intr, wh, hand, pix_off, vi);
        const float* hv32 = v32 + (size_t)3 * V * c.hand;
        const double* hv64 = verts + (size_t)3 * V * c.hand;
        const double* hn = normals + (size_t)3 * V * c.hand;
        const double* tex = albedo + (size_t)3 * th * tw * c.hand;
        double* gv = g_verts + (size_t)3 * V * c.hand;
        view_edges(&c, hv32, faces, E, edges, edge_faces, ed);
        uint64_t Tlen = 0;
        for (int e = 0; e < E; ++e) Tlen += ed[e].w;
        if (Tlen == 0) continue;
        if (wq)   /* sampling weights: length weights replaced where sampled */
            for (int e = 0; e < E; ++e)
                if (ed[e].w > 0) ed[e].w = wq[(size_t)vi * E + e];
        uint64_t T = 0;
        for (int e = 0; e < E; ++e) { T += ed[e].w; cdf[e] = T; }
        int64_t Mv = (int64_t)((Tlen + 255) / 256);
        if (budget_override) Mv = budget_override[vi];
        if (Mv <= 0) continue;
        for (int64_t k = 0; k < Mv; ++k) {
            uint64_t ctr[4] = {(uint64_t)k, 0, (uint64_t)(uint32_t)vi | (DOMAIN_EDGE << 32), (uint64_t)iter};
            uint64_t key[2] = {seed, 0};
            uint64_t r[4];
            philox4x64_10(ctr, key, r);
            /* stratum k of the quantised-length CDF: targets [k T / M, (k+1) T / M) */
            uint64_t lo = (uint64_t)(((unsigned __int128)k * T) / (uint64_t)Mv);
            uint64_t hi = (uint64_t)(((unsigned __int128)(k + 1) * T) / (uint64_t)Mv);
            uint64_t width = hi - lo;
            if (width == 0) continue;
            uint64_t target = lo + (uint64_t)(((unsigned __int128)r[0] * width) >> 64);
            /* first edge whose inclusive prefix sum exceeds the target */
            int e = 0;
            while (cdf[e] <= target) ++e;
            const edge32_t* q = ed + e;
            float u = u24_hi(r[1]);
            float t = q->t0 + u * (q->t1 - q->t0);
            float dx = q->bx - q->ax, dy = q->by - q->ay;
            float x = q->ax + t * dx;
            float y = q->ay + t * dy;
            float len = sqrtf(dx * dx + dy * dy);
            float nhx = dy / len, nhy = -dx / len;
            float xp = x + delta * nhx, yp = y + delta * nhy;
            float xm = x - delta * nhx, ym = y - delta * nhy;
            int px = (int)floorf(x), py = (int)floorf(y);
            if (px < 0) px = 0;
            if (px > c.W - 1) px = c.W - 1;
            if (py < 0) py = 0;
            if (py > c.H - 1) py = c.H - 1;
            int64_t pix = c.pix0 + (int64_t)py * c.W + px;
            const double* g = dimage + 3 * pix;
            const double* bg = background + 3 * pix;
            double cp[3], cm[3];
            hit_t h;
            if (trace_point(&c, &m, hv32, hv64, xp, yp, xp, yp, &h) >= 0) {
                shade_t S; shade_point(&m, hn, tex, &h, &S);
                for (int ch = 0; ch < 3; ++ch) cp[ch] = S.col[ch];
            } else {
                for (int ch = 0; ch < 3; ++ch) cp[ch] = bg[ch];
            }
            if (trace_point(&c, &m, hv32, hv64, xm, ym, xm, ym, &h) >= 0) {
                shade_t S; shade_point(&m, hn, tex, &h, &S);
                for (int ch = 0; ch < 3; ++ch) cm[ch] = S.col[ch];
            } else {
                for (int ch = 0; ch < 3; ++ch) cm[ch] = bg[ch];
            }
            int a = edges[2 * e], b = edges[2 * e + 1];
            double pa[2], pb[2], Ja[2][3], Jb[2][3];
            project64(&c, hv64 + 3 * a, pa, Ja);
            project64(&c, hv64 + 3 * b, pb, Jb);
            double ddx = pb[0] - pa[0], ddy = pb[1] - pa[1];
            double len64 = sqrt(ddx * ddx + ddy * ddy);
            double nx = ddy / len64, ny = -ddx / len64;
            double ell = len64 * ((double)q->t1 - (double)q->t0);
            /* sample weight: (stratum probability width/T) / (pdf (w_e/T)/ell) */
            double inv_pdf_m = ell * (double)width / (double)q->w;
            double jump = g[0] * (cm[0] - cp[0]) + g[1] * (cm[1] - cp[1]) + g[2] * (cm[2] - cp[2]);
            double s = jump * inv_pdf_m;
            if (edge_stats) edge_stats[(size_t)vi * E + e] += fabs(s);
            if (dc_stats && (g[0] != 0.0 || g[1] != 0.0 || g[2] != 0.0)) {
                double* d = dc_stats + ((size_t)vi * E + e) * 4;
                for (int ch = 0; ch < 3; ++ch) d[ch] += fabs(cm[ch] - cp[ch]);
                d[3] += 1.0;
            }
            double td = (double)t;
            double dpa[2] = {(1.0 - td) * s * nx, (1.0 - td) * s * ny};
            double dpb[2] = {td * s * nx, td * s * ny};
            for (int k3 = 0; k3 < 3; ++k3) {
                gv[3 * a + k3] += Ja[0][k3] * dpa[0] + Ja[1][k3] * dpa[1];
                gv[3 * b + k3] += Jb[0][k3] * dpb[0] + Jb[1][k3] * dpb[1];
            }
        }
    }
    free(cdf);
    free(ed);
    free(v32);
}

/* ------------------------------------------------------------------------ */
/* single-ray queries (for pins of the intersection decision)                */
/* ------------------------------------------------------------------------ */

/* closest hit of explicit float32 rays against a triangle soup */
void ora_trace_rays32(int n_rays, const float* org, const float* dir, int V, const float* v32,
                      int F, const int32_t* faces, int32_t* face_out, float* t_out)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n_rays; ++i) {
        ray32_t r;
        for (int k = 0; k < 3; ++k) { r.o[k] = org[3 * i + k]; r.d[k] = dir[3 * i + k]; }
        ray32_setup(&r);
        int best = -1;
        float tb = INFINITY;
        for (int f = 0; f < F; ++f) {
            const int32_t* tri = faces + 3 * f;
            float t;
            if (watertight32(&r, v32 + 3 * tri[0], v32 + 3 * tri[1], v32 + 3 * tri[2], &t))
                if (t < tb) { tb = t; best = f; }
        }
        face_out[i] = best;
        t_out[i] = tb;
    }
    (void)V;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
