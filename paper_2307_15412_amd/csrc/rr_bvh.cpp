// rr_bvh.cpp -- host construction of the two-wide BVH used by the tracer.
//
// Binned surface-area-heuristic splits (16 bins per axis) with leaves of up
// to 4 triangles (8 when a split does not pay off).  When the remaining depth
// budget gets tight the builder switches to object-median splits, which
// bounds the depth by 31 so that the per-lane LDS stack of 32 entries can
// never overflow.  Child boxes are stored in the parent, rounded outward to
// float and padded by 1 mm plus 1e-6 of the scene extent: the FP32 slab test
// on the device can therefore only over-include, never miss a triangle that
// the FP64 intersection test would accept.  Leaf triangles are stored in leaf
// order as 12 words: 9 vertex coordinates, the triangle's upload index, its
// object and its material mix alpha.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

#include "rr_internal.h"

namespace {

struct Prim {
    float lo[3], hi[3], c[3];
};

struct Box {
    float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX};
    float hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    void grow(const float *l, const float *h)
    {
        for (int a = 0; a < 3; a++) {
            lo[a] = std::min(lo[a], l[a]);
            hi[a] = std::max(hi[a], h[a]);
        }
    }
    double area() const
    {
        double dx = std::max(0.0f, hi[0] - lo[0]), dy = std::max(0.0f, hi[1] - lo[1]),
               dz = std::max(0.0f, hi[2] - lo[2]);
        return dx * dy + dy * dz + dz * dx;
    }
};

int ceil_log2(int64_t n)
{
    int l = 0;
    while ((int64_t(1) << l) < n) l++;
    return l;
}

struct Builder {
    std::vector<Prim> prims;
    std::vector<int64_t> idx;
    std::vector<float> nodes;
    double pad = 1e-3;
    int max_depth = 0;

    static int32_t leaf_ref(int64_t first, int64_t count)
    {
        return ~(int32_t)((first << 3) | (count - 1));
    }

    void write_box(float *dst, const Box &b) const
    {
        for (int a = 0; a < 3; a++) {
            float lo = (float)((double)b.lo[a] - pad);
            if ((double)lo > (double)b.lo[a] - pad) lo = std::nextafter(lo, -FLT_MAX);
            float hi = (float)((double)b.hi[a] + pad);
            if ((double)hi < (double)b.hi[a] + pad) hi = std::nextafter(hi, FLT_MAX);
            dst[a] = lo;
            dst[3 + a] = hi;
        }
    }

    int64_t new_node()
    {
        int64_t n = (int64_t)nodes.size() / 16;
        nodes.resize(nodes.size() + 16, 0.0f);
        return n;
    }

    void set_node(int64_t n, const Box &b0, int32_t r0, const Box &b1, int32_t r1)
    {
        float bx0[6], bx1[6];
        write_box(bx0, b0);
        write_box(bx1, b1);
        float *N = &nodes[16 * n];
        // (lo0.xyz, hi0.x) (hi0.yz, lo1.xy) (lo1.z, hi1.xyz) (ref0, ref1, 0, 0)
        N[0] = bx0[0]; N[1] = bx0[1]; N[2] = bx0[2]; N[3] = bx0[3];
        N[4] = bx0[4]; N[5] = bx0[5]; N[6] = bx1[0]; N[7] = bx1[1];
        N[8] = bx1[2]; N[9] = bx1[3]; N[10] = bx1[4]; N[11] = bx1[5];
        std::memcpy(&N[12], &r0, 4);
        std::memcpy(&N[13], &r1, 4);
        N[14] = 0.0f;
        N[15] = 0.0f;
    }

    Box range_box(int64_t b, int64_t e) const
    {
        Box bx;
        for (int64_t k = b; k < e; k++) bx.grow(prims[idx[k]].lo, prims[idx[k]].hi);
        return bx;
    }

    // Build [b, e) at `depth`; returns the child reference, box in *out.
    int32_t build(int64_t b, int64_t e, int depth, Box *out)
    {
        const int64_t n = e - b;
        Box bx = range_box(b, e);
        *out = bx;
        if (n <= 4) {
            max_depth = std::max(max_depth, depth);
            return leaf_ref(b, n);
        }
        Box cb;
        for (int64_t k = b; k < e; k++) cb.grow(prims[idx[k]].c, prims[idx[k]].c);
        int axis = 0;
        for (int a = 1; a < 3; a++)
            if (cb.hi[a] - cb.lo[a] > cb.hi[axis] - cb.lo[axis]) axis = a;
        const bool degenerate = !(cb.hi[axis] > cb.lo[axis]);
        const bool force_median = degenerate || depth + ceil_log2((n + 3) / 4) >= 30;
        int64_t mid = -1;
        if (!force_median) {
            const int NB = 16;
            double best_cost = INFINITY;
            int best_axis = -1, best_split = -1;
            for (int a = 0; a < 3; a++) {
                float ext = cb.hi[a] - cb.lo[a];
                if (!(ext > 0.0f)) continue;
                Box bins[NB];
                int64_t cnt[NB] = {0};
                const float scale = (float)NB / ext;
                for (int64_t k = b; k < e; k++) {
                    const Prim &p = prims[idx[k]];
                    int bi = std::min(NB - 1, (int)((p.c[a] - cb.lo[a]) * scale));
                    bins[bi].grow(p.lo, p.hi);
                    cnt[bi]++;
                }
                Box lacc[NB];
                int64_t lcnt[NB];
                Box acc;
                int64_t c = 0;
                for (int i = 0; i < NB; i++) {
                    if (cnt[i]) acc.grow(bins[i].lo, bins[i].hi);
                    c += cnt[i];
                    lacc[i] = acc;
                    lcnt[i] = c;
                }
                Box racc;
                int64_t rc = 0;
                for (int i = NB - 1; i > 0; i--) {
                    if (cnt[i]) racc.grow(bins[i].lo, bins[i].hi);
                    rc += cnt[i];
                    int64_t lc = lcnt[i - 1];
                    if (lc == 0 || rc == 0) continue;
                    double cost = lacc[i - 1].area() * (double)lc + racc.area() * (double)rc;
                    if (cost < best_cost) {
                        best_cost = cost;
                        best_axis = a;
                        best_split = i;
                    }
                }
            }
            const double leaf_cost = bx.area() * (double)n;
            if (best_axis < 0 || (n <= RR_LEAF_MAX && best_cost >= leaf_cost)) {
                if (n <= RR_LEAF_MAX) {
                    max_depth = std::max(max_depth, depth);
                    return leaf_ref(b, n);
                }
            }
            if (best_axis >= 0) {
                const float ext = cb.hi[best_axis] - cb.lo[best_axis];
                const float scale = (float)NB / ext;
                const float lo = cb.lo[best_axis];
                auto it = std::partition(idx.begin() + b, idx.begin() + e, [&](int64_t i) {
                    int bi = std::min(NB - 1, (int)((prims[i].c[best_axis] - lo) * scale));
                    return bi < best_split;
                });
                mid = it - idx.begin();
                if (mid == b || mid == e) mid = -1;
            }
        }
        if (mid < 0) {
            mid = b + n / 2;
            if (!degenerate) {
                std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e,
                                 [&](int64_t i, int64_t j) {
                                     if (prims[i].c[axis] != prims[j].c[axis])
                                         return prims[i].c[axis] < prims[j].c[axis];
                                     return i < j;
                                 });
            }
        }
        int64_t me = new_node();
        Box lb, rb;
        int32_t l = build(b, mid, depth + 1, &lb);
        int32_t r = build(mid, e, depth + 1, &rb);
        set_node(me, lb, l, rb, r);
        return (int32_t)me;
    }
};

}  // namespace

int rr_build_bvh(const float *verts, int64_t nv, const int32_t *tris, const int32_t *tri_obj,
                 const float *obj_alpha, int64_t nt, HostBvh &out, std::string &err)
{
    out.nodes.clear();
    out.tris.clear();
    out.depth = 0;
    if (nt == 0) return 0;
    if (nt >= (int64_t(1) << 27)) {
        err = "too many triangles for the leaf encoding";
        return RR_EUNSUPPORTED;
    }
    Builder B;
    B.prims.resize(nt);
    double maxabs = 0.0;
    for (int64_t i = 0; i < nt; i++) {
        Prim &p = B.prims[i];
        for (int a = 0; a < 3; a++) {
            p.lo[a] = FLT_MAX;
            p.hi[a] = -FLT_MAX;
        }
        for (int c = 0; c < 3; c++) {
            const float *v = verts + 3 * (int64_t)tris[3 * i + c];
            for (int a = 0; a < 3; a++) {
                p.lo[a] = std::min(p.lo[a], v[a]);
                p.hi[a] = std::max(p.hi[a], v[a]);
                maxabs = std::max(maxabs, (double)std::fabs(v[a]));
            }
        }
        for (int a = 0; a < 3; a++) p.c[a] = 0.5f * (p.lo[a] + p.hi[a]);
    }
    (void)nv;
    B.pad = 1e-3 + 1e-6 * maxabs;
    B.idx.resize(nt);
    for (int64_t i = 0; i < nt; i++) B.idx[i] = i;
    B.nodes.reserve((size_t)(2 * nt / 4 + 16) * 16);
    Box rootbox;
    int64_t root = B.new_node();
    int32_t r = B.build(0, nt, 1, &rootbox);
    if (r >= 0) {
        // copy the root's contents into node 0
        int64_t n = r;
        std::copy(B.nodes.begin() + 16 * n, B.nodes.begin() + 16 * n + 16, B.nodes.begin());
        // node r is now unreferenced (harmless)
    } else {
        // a single leaf: node 0 holds it twice, the second copy behind a far box
        Box far;
        for (int a = 0; a < 3; a++) far.lo[a] = far.hi[a] = 1e30f;
        B.set_node(root, rootbox, r, far, r);
    }
    if (B.max_depth > RR_STACK - 1) {
        err = "BVH depth bound violated";
        return RR_EINVAL;
    }
    out.depth = B.max_depth;
    out.nodes.swap(B.nodes);
    out.tris.resize((size_t)nt * 12);
    for (int64_t k = 0; k < nt; k++) {
        int64_t i = B.idx[k];
        float *T = &out.tris[12 * k];
        for (int c = 0; c < 3; c++) {
            const float *v = verts + 3 * (int64_t)tris[3 * i + c];
            T[3 * c + 0] = v[0];
            T[3 * c + 1] = v[1];
            T[3 * c + 2] = v[2];
        }
        int32_t id = (int32_t)i, ob = tri_obj[i];
        std::memcpy(&T[9], &id, 4);
        std::memcpy(&T[10], &ob, 4);
        T[11] = obj_alpha[ob];   // the face's material mix (Eq. 3), replaceable per face
    }
    return 0;
}
