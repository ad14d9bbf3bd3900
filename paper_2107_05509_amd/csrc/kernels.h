// Kernel argument records of the handrt library (device pointers only).
#pragma once

#include "device.h"

namespace hr {

constexpr int kMaxJoints = 32;
constexpr int kMaxShape = 16;
constexpr int kMaxInfl = 8;     // skinning weights per vertex
constexpr int kSkinPart = 12 + 12 * kMaxJoints + 16;   // per-hand sums of the skinning backward
constexpr int kVfSlots = 12;    // faces per vertex in the corner table (more: the CSR list)
constexpr int kLossChunk = 4096;     // pixels per loss block (never straddles views)
constexpr int kCounts = 18;          // work counters: 6 per ray-tracing kernel (render, interior adjoint, edges)

struct MeshDev {
    int V, F, J, K, E;
    const float* v_template;   // [3,V]
    const float* shapedirs;    // [K,3,V]
    const float* j_regressor;  // [J,V]
    const float* weights;      // [V,J]
    const int* parents;        // [J]
    const int* faces;          // [F,3]
    const float* uv;           // [V,2]
    const int* edges;          // [E,2]
    const int* edge_faces;     // [E,2]
    const int4* edge_verts;    // [E,2] (va, vb, face 0's vertices, face 1's vertices or -1)
    const int* vf_off;         // [V+1]
    const int* vf_faces;       // [3F]
    const int4* vf_corner;     // [kVfSlots,V] the first kVfSlots faces around each vertex as
                               // (a, b, c, face), padded with (v, v, v, 0)
    const float* jt;           // [J,3] J_reg T: rest joints of the template
    const float* js;           // [J,3,K] J_reg S: joint displacement per shape coefficient
    const double* jt64;        // the same two tables in float64 (the forward skinning)
    const double* js64;
    const int* jdepth;         // [J] depth in the joint tree (root 0)
    int max_depth;
    int infl;                  // skinning weights per vertex (padded with weight 0)
    const int* widx;           // [infl,V] joint of each weight
    const float* wval;         // [infl,V]
};

// Topology of each hand's hierarchy (bounds are refit every iteration).
// Arrays are per hand with fixed strides.
struct BvhDev {
    int node_stride;           // >= internal nodes of any hand
    int level_stride;          // >= levels + 1 of any hand
    const int* n_levels;       // [H]
    const int* child;          // [H, node_stride, 2] child codes
    const int* perm;           // [H, F] face of each leaf slot
    const int* order;          // [H, node_stride] internal nodes sorted by height (the traversal's
                               // numbering puts them at n - 1 - position: the root is 0)
    const int* level_off;      // [H, level_stride] offsets into order per height
    const int* slot_verts;     // [H, F, 3] vertex ids of each leaf slot's triangle
};

// Per-view screen bins of the camera rays: each bin of 2^log2 x 2^log2
// pixels (16 x 16 by default) lists the leaf slots of the triangles whose
// padded screen bounds touch it.  Camera
// rays all start at the camera centre, so a ray through a screen point can
// only hit triangles listed in that point's bin: the lists replace the
// hierarchy for them (views whose bins are incomplete keep the hierarchy).
struct BinDev {
    int* count;                // [bins of all views] triangles listed per bin
    int* off;                  // [bins of all views] first entry of the bin in its view's entries
    uint16_t* entries;         // [n_views, cap] leaf slots, bin after bin
    float4* box;               // [n_views, F] padded screen bounds (x0, y0, x1, y1) per leaf slot
    int* binned;               // [n_views] 1: the view's bins are complete and valid
    int cap;                   // entries per view
    int log2;                  // bins of 2^log2 x 2^log2 pixels (kMinBinLog2 .. kMaxBinLog2)
};

// wave tiles: a tile of 2^tw_log2 x 2^th_log2 pixels, 2^spp_log2 lanes per
// pixel (64 lanes per wave); spp > 64 takes `rounds` passes of 64 samples
struct TileShape {
    int spp_log2, tw_log2, th_log2, rounds;
};

struct RenderArgs {
    const int2* tiles;         // (view, tx | ty << 16)
    const int* tile_count;
    TileShape ts;
    const ViewDev* views;
    const Node* nodes;
    const Tri* tris;
    const float* normals;
    const float* uv;
    const float* albedo;
    const float* background;
    float* image;
    int* hit_face;
    uint64_t* hit_rec;         // [tiles, rounds, 64] each sample's random word and hit leaf slot (hit_record), for the adjoint
    int* hit_iter;             // iteration of the stored hits
    const int4* view_rect;     // nullable: [n_views] pixel rectangle of each view's tiles; pixels
                               // outside it are set to the background by the render blocks
    int n_views;
    float* clear[3];           // nullable: buffers the render blocks zero (a following backward's accumulators)
    long long clear_n[3];
    float* dimage;             // nullable: [P,3] L1 loss gradient written with the image (needs view_rect)
    const float* target;       // [P,3] with dimage
    const uint8_t* mask;       // [P] nullable
    const float* view_scale;   // [n_views] 1 / (3 * masked pixels), with dimage
    unsigned long long* counts;   // [6] counting variant: rays traced, node visits, triangle tests, hits,
                                  // packet node visits and packet triangle tests (TraceCount)
    BinDev bins;               // screen bins of the camera rays
    int n_nodes, n_faces, n_verts, tex_h, tex_w, spp;
    uint32_t iter;
    const int* iter_dev;       // nullable: iteration index read on the device instead of `iter`
    uint64_t seed;
    Shading shading;
};

struct AdjointArgs {
    const int2* tiles;
    const int* tile_count;
    TileShape ts;
    const ViewDev* views;
    const int* faces;
    const Node* nodes;
    const Tri* tris;
    const float* normals;
    const float* uv;
    const float* albedo;
    const float* dimage;
    float* grad_albedo;
    float* gface;              // [hands,F,18] per-triangle corner gradients
    const uint64_t* hit_rec;   // nullable: sample records stored by the render of the same geometry
    const int* hit_iter;
    unsigned long long* counts;
    int n_nodes, n_faces, n_verts, tex_h, tex_w, spp;
    uint32_t iter;
    const int* iter_dev;       // nullable: iteration index read on the device instead of `iter`
    uint64_t seed;
    Shading shading;
};

struct LossArgs {
    const int2* chunks;        // (view, first pixel)
    const ViewDev* views;
    const float* image;        // nullable: masked-pixel counts only
    const float* target;
    const uint8_t* mask;
    float* partial;            // [n_chunks,2]
    const int* view_chunk_off; // [n_views+1]
    const int* hand_view_off;  // [n_hands+1]
    const int* hand_views;     // [n_views]
    float* view_scale;         // [n_views] nullable (not written)
    float* loss;               // [n_hands] nullable (not written)
    float* dimage;
    int n_hands;
};

// one stored edge sample (see edge_samples)
struct alignas(16) EdgeSample {
    int vi, e;                 // view and edge; vi < 0: empty stratum
    long long pg;              // packed pixel owning the sample point
    float t, wgt;              // position along the edge, stratum width over sampling weight
    float dc[3];               // c(x - delta n) - c(x + delta n)
    float pad;
};

struct EdgeArgs {
    MeshDev m;
    const ViewDev* views;
    const float* verts;
    EdgeRec* rec;              // [n_views,E]
    unsigned long long* cdf;   // [n_views,E]
    unsigned long long* total; // [n_views]
    long long* budget;         // [n_views]
    int budget_div;            // quantised length (1/256 px) per edge sample: budget = ceil(total / budget_div)
    long long* prefix;         // [n_views+1] exclusive prefix of budgets
    int n_views;

    const Node* nodes;
    const Tri* tris;
    const float* normals;
    const float* uv;
    const float* albedo;
    const float* background;
    const float* dimage;
    float* gacc;               // [views,V,3] float64 vertex-gradient slots (6 floats of storage per vertex)
    float* stat_a;             // [n_views,E] nullable: sum of |sample contribution| per edge
    float* stat_dc;            // [n_views,E,4] nullable: sum of |c- - c+| per channel, sample count
    EdgeSample* samples;       // [sample_cap] traced samples
    long long sample_cap;
    int few_waves;             // the device's compute units: the few-tile render's edge packets shrink
                               // while their waves stay at most this many
    unsigned long long* counts;
    int n_nodes, tex_h, tex_w;
    float delta;
    uint32_t iter;
    const int* iter_dev;       // nullable: iteration index read on the device instead of `iter`
    uint64_t seed;
    Shading shading;
};

struct AdamArgs {
    float* params;
    float* albedo;
    const float* grad_params;
    const float* grad_albedo;
    float *m_params, *v_params, *m_albedo, *v_albedo;
    long long n_albedo;
    int n_hands;
    float lr[6];
    float beta1, beta2, eps, bc1, bc2;
    const int* iter_dev;       // nullable: step count = *iter_dev + 1, bias corrections on the device
};

// one launch of geometry preparation (k_prepare)
struct PrepArgs {
    MeshDev m;
    BvhDev b;
    const float* verts;
    float* normals;
    Tri* tris;
    Node* nodes;
    EdgeArgs e;                // with_setup: the silhouette tables
    const ViewDev* views;
    TileShape ts;
    int2* tiles;
    int* tile_count;           // zero before the launch
    int4* view_rect;
    const uint8_t* mask;       // with_scale (nullable: all pixels)
    float* view_scale;
    int* setup_done;           // with_setup: finished silhouette tables (zero between launches)
    BinDev bins;               // the views' screen bins (built every launch)
    int with_bins;             // 0: every view marked unbinned (hierarchy only)
    int n_hands, n_views, with_setup, with_scale;
    float* bvh_cost;           // [H] the refitted hierarchy's traversal cost (see refit_hand)
};

// geometry backward (k_geom_p1, k_geom_p2)
struct GeomBwdArgs {
    MeshDev m;
    const float* params;       // [H,64]
    const float* verts;        // [H,V,3]
    const float* gacc;         // [views,V,3] float64 per-vertex slots of each view (edge term)
    const int* hand_view_off;  // [H+1] views of each hand
    const int* hand_views;
    const float* gface;        // [H,F,18] triangle-corner slots (interior term)
    float* grad_verts;         // nullable [H,V,3]
    float* grad_normals;       // nullable [H,V,3]
    float* grad_params;        // [H,64]
    AdamArgs adam;             // with adam_params: the parameters' step
    int adam_params;
    LossArgs loss;             // with_loss: the hand's loss value from the chunk partials
    int with_loss;
    float* gr;                 // [H,V,3] dL/d(raw vertex normal) (first launch -> second)
    float* gpos;               // [H,V,3] dL/dv from the slots
    float* part;               // [H, kSkinPart] the skinning sums (atomic; zero between launches)
    int* counter;              // [H] finished blocks (zero between launches)
    const float* js_saved;     // nullable: [H, joint state] left by the skinning of the same parameters
    int n_hands;
    int p1_blocks;             // vertex blocks per hand of the first launch
    int* iter_advance;         // nullable: iteration counter, incremented once every hand has finished
    int* hand_counter;         // [1] finished hands (zero between launches)
    const float* prior_target; // nullable: [H,J,3] target joints of the joint prior
    float prior_lambda;        // its weight
    float prior_gamma;         // its smooth-L1 threshold (model units)
};

}  // namespace hr
