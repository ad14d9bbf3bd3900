// Host-side construction of the topology of a binary bounding-volume
// hierarchy over triangles (bounds are refit on the device every iteration).
#pragma once

#include <algorithm>
#include <numeric>
#include <vector>

namespace hr {

struct HostBvh {
    std::vector<int> child;      // [n,2]
    std::vector<int> perm;       // [F]
    std::vector<int> order, level_off;
    int depth = 0;
};

inline int leaf_code(int start, int count) { return ~((start << 3) | count); }

struct Box {
    float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
    void grow(const float* p) { for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], p[k]); hi[k] = std::max(hi[k], p[k]); } }
    bool empty() const { return lo[0] > hi[0]; }
    void grow(const Box& b)
    {
        if (b.empty()) return;
        grow(b.lo);
        grow(b.hi);
    }
    float area() const
    {
        float d[3];
        for (int k = 0; k < 3; ++k) d[k] = std::max(0.0f, hi[k] - lo[k]);
        return 2.0f * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
    }
};

// Binned surface-area-heuristic build (16 bins per axis over centroid bounds),
// leaves of at most leaf_max triangles; nodes in depth-first order.
struct SahBuilder {
    HostBvh& b;
    std::vector<int>& idx;
    const std::vector<Box>& tb;
    const std::vector<float>& cen;
    int leaf_max;

    int build(int lo, int hi, int depth)
    {
        b.depth = std::max(b.depth, depth);
        const int node = (int)b.child.size() / 2;
        b.child.push_back(0);
        b.child.push_back(0);
        const int n = hi - lo;
        Box cb;
        for (int i = lo; i < hi; ++i) cb.grow(&cen[3 * idx[i]]);
        constexpr int NB = 16;
        float best_cost = 1e30f;
        int best_axis = -1, best_bin = -1;
        for (int ax = 0; ax < 3; ++ax) {
            const float ext = cb.hi[ax] - cb.lo[ax];
            if (!(ext > 0.0f)) continue;
            Box bins[NB];
            int cnt[NB] = {0};
            for (int i = lo; i < hi; ++i) {
                int k = (int)((cen[3 * idx[i] + ax] - cb.lo[ax]) / ext * NB);
                k = std::min(std::max(k, 0), NB - 1);
                bins[k].grow(tb[idx[i]]);
                cnt[k]++;
            }
            float right_area[NB];
            int right_cnt[NB];
            Box acc;
            int c = 0;
            for (int k = NB - 1; k > 0; --k) {
                acc.grow(bins[k]);
                c += cnt[k];
                right_area[k] = acc.area();
                right_cnt[k] = c;
            }
            Box lacc;
            int lc = 0;
            for (int k = 0; k < NB - 1; ++k) {
                lacc.grow(bins[k]);
                lc += cnt[k];
                if (lc == 0 || right_cnt[k + 1] == 0) continue;
                const float cost = lacc.area() * lc + right_area[k + 1] * right_cnt[k + 1];
                if (cost < best_cost) { best_cost = cost; best_axis = ax; best_bin = k; }
            }
        }
        int mid;
        if (best_axis < 0) {
            mid = (lo + hi) / 2;   // all centroids coincide: any split
        } else {
            const float ext = cb.hi[best_axis] - cb.lo[best_axis];
            auto it = std::partition(idx.begin() + lo, idx.begin() + hi, [&](int t) {
                int k = (int)((cen[3 * t + best_axis] - cb.lo[best_axis]) / ext * NB);
                k = std::min(std::max(k, 0), NB - 1);
                return k <= best_bin;
            });
            mid = (int)(it - idx.begin());
            if (mid == lo || mid == hi) mid = (lo + hi) / 2;
        }
        const int ranges[2][2] = {{lo, mid}, {mid, hi}};
        for (int c = 0; c < 2; ++c) {
            const int a = ranges[c][0], e = ranges[c][1];
            const int code = (e - a <= leaf_max) ? leaf_code(a, e - a) : build(a, e, depth + 1);
            b.child[2 * node + c] = code;
        }
        (void)n;
        return node;
    }
};

inline HostBvh build_bvh(const float* verts, const int* faces, int F, int leaf_max)
{
    HostBvh b;
    std::vector<Box> tb(F);
    std::vector<float> cen(3 * F);
    for (int f = 0; f < F; ++f) {
        for (int k = 0; k < 3; ++k) tb[f].grow(verts + 3 * faces[3 * f + k]);
        for (int k = 0; k < 3; ++k) cen[3 * f + k] = 0.5f * (tb[f].lo[k] + tb[f].hi[k]);
    }
    std::vector<int> idx(F);
    std::iota(idx.begin(), idx.end(), 0);
    if (F <= leaf_max) {
        b.child = {leaf_code(0, F), leaf_code(0, 0)};
    } else {
        SahBuilder sb{b, idx, tb, cen, leaf_max};
        sb.build(0, F, 1);
    }
    b.perm = idx;
    const int n = (int)b.child.size() / 2;
    // heights: leaves 0; a node is refit after all its children
    std::vector<int> height(n, 0);
    for (int i = n - 1; i >= 0; --i) {   // children have larger indices (preorder)
        int h = 1;
        for (int c = 0; c < 2; ++c) {
            int code = b.child[2 * i + c];
            if (code >= 0) h = std::max(h, height[code] + 1);
        }
        height[i] = h;
    }
    int maxh = *std::max_element(height.begin(), height.end());
    b.level_off.assign(maxh + 1, 0);
    for (int L = 1; L <= maxh; ++L) {
        for (int i = 0; i < n; ++i)
            if (height[i] == L) b.order.push_back(i);
        b.level_off[L] = (int)b.order.size();
    }
    return b;
}


}  // namespace hr
