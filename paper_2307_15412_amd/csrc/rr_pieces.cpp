// rr_pieces.cpp -- pieces of the per-triangle launch.
//
// Every triangle, in upload order, is cut by midpoint subdivision into four
// while the piece subtends more than omega_max steradians from the Tx phase
// centre and its depth is below depth_max; children are taken in the order
// (v0, m01, m20), (m01, v1, m12), (m20, m12, v2), (m01, m12, m20), depth
// first.  Pieces none of whose rays can enter the field of view are dropped
// (all three vertices beyond the same bounding plane of the azimuth wedge,
// or inside the same excluded elevation cone where that cone is convex, by a
// margin of 1e-9 of their distance, as seen from every source).  Each piece
// keeps its parent triangle (the one its rays must hit first).  omega_max = 0
// gives the triangles in view.  The subdivision
// only moves rays towards triangles that fill much solid angle (a near-field
// ground plane); every ray is weighted by its own piece's area, so the
// estimate stays unbiased for any subdivision.  Built in FP64 on the host
// (midpoints of FP32 vertices are exact); this file is compiled without
// floating-point contraction so that the threshold decisions are those of the
// plain IEEE expressions.
#include <cmath>

#include "rr_internal.h"

namespace {

struct V3 {
    double x, y, z;
};

V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double len(V3 a) { return std::sqrt(dot(a, a)); }
V3 midp(V3 a, V3 b) { return {(a.x + b.x) * 0.5, (a.y + b.y) * 0.5, (a.z + b.z) * 0.5}; }

// solid angle of triangle (a, b, c) seen from o (Van Oosterom and Strackee 1983)
double solid_angle(V3 a, V3 b, V3 c, V3 o)
{
    const V3 x = sub(a, o), y = sub(b, o), z = sub(c, o);
    const double lx = len(x), ly = len(y), lz = len(z);
    const double num = std::fabs(dot(x, cross(y, z)));
    const double den = lx * ly * lz + dot(x, y) * lz + dot(x, z) * ly + dot(y, z) * lx;
    return 2.0 * std::atan2(num, den);
}

const double CULL_EPS = 1e-9;

bool beyond_fov(V3 a, V3 b, V3 c, V3 src, const RrFov &f)
{
    const V3 r[3] = {sub(a, src), sub(b, src), sub(c, src)};
    int n0 = 0, n1 = 0, n2 = 0, n3 = 0;
    for (int k = 0; k < 3; k++) {
        const double l = len(r[k]);
        if (f.c0 * r[k].y - f.s0 * r[k].x < -CULL_EPS * l) n0++;
        if (f.c1 * r[k].y - f.s1 * r[k].x > CULL_EPS * l) n1++;
        if (r[k].z < f.slo * l - CULL_EPS * l) n2++;
        if (r[k].z > f.shi * l + CULL_EPS * l) n3++;
    }
    return n0 == 3 || n1 == 3 || (f.slo <= 0.0 && n2 == 3) || (f.shi >= 0.0 && n3 == 3);
}

bool outside_fov(V3 a, V3 b, V3 c, const RrFov &f)
{
    for (int32_t t = 0; t < f.n_src; t++)
        if (!beyond_fov(a, b, c, {f.src[3 * t], f.src[3 * t + 1], f.src[3 * t + 2]}, f))
            return false;
    return true;
}

struct Cutter {
    V3 o;
    double omega_max;
    int depth_max;
    int64_t limit;
    const RrFov *fov;
    std::vector<double> &verts;
    std::vector<int32_t> &parent;

    bool cut(V3 a, V3 b, V3 c, int32_t par, int depth)
    {
        if (omega_max > 0.0 && depth < depth_max && solid_angle(a, b, c, o) > omega_max) {
            const V3 ab = midp(a, b), bc = midp(b, c), ca = midp(c, a);
            return cut(a, ab, ca, par, depth + 1) && cut(ab, b, bc, par, depth + 1) &&
                   cut(ca, bc, c, par, depth + 1) && cut(ab, bc, ca, par, depth + 1);
        }
        if (fov && outside_fov(a, b, c, *fov)) return true;
        if ((int64_t)parent.size() >= limit) return false;
        const V3 v[3] = {a, b, c};
        for (int k = 0; k < 3; k++) {
            verts.push_back(v[k].x);
            verts.push_back(v[k].y);
            verts.push_back(v[k].z);
        }
        parent.push_back(par);
        return true;
    }
};

}  // namespace

int rr_build_pieces(const float *verts, const int32_t *tris, int64_t n_tris, const double *o,
                    double omega_max, int depth_max, const RrFov *fov, int64_t limit,
                    std::vector<double> &pverts, std::vector<int32_t> &parent)
{
    pverts.clear();
    parent.clear();
    Cutter C{{o[0], o[1], o[2]}, omega_max, depth_max, limit, fov, pverts, parent};
    for (int64_t f = 0; f < n_tris; f++) {
        V3 v[3];
        for (int k = 0; k < 3; k++) {
            const float *p = verts + 3 * (int64_t)tris[3 * f + k];
            v[k] = {(double)p[0], (double)p[1], (double)p[2]};
        }
        if (!C.cut(v[0], v[1], v[2], (int32_t)f, 0)) return RR_EOVERFLOW;
    }
    return RR_OK;
}
