// k_trace.hip -- ray generation, BVH traversal, FP64 intersection, material
// bounce, reception and path bookkeeping for gfx950.
//
// One lane carries one ray through all of its bounces (Section III-A: each
// transmitter sends out many rays; Eqs. 1-3 give the outgoing direction at
// each hit; Section III-B: received rays keep their total path length).
// Box tests run in FP32 against boxes the builder padded outward, so they can
// only over-include; every triangle decision (Moller-Trumbore) and every
// length, bounce and reception computation runs in FP64 with no FMA
// contraction, which makes the closest-hit ids identical to a plain FP64
// evaluation of the same formulas.  The per-lane BVH stack lives in LDS,
// laid out [depth][lane] so that lanes at the same depth hit distinct banks.
// Received paths are appended with one atomic per wavefront and later put in
// (virtual ray, bounce) order by a scan over per-ray counts and a scatter,
// so the result does not depend on atomic ordering.
#include <algorithm>

#include "rr_internal.h"

#pragma clang fp contract(off)

namespace {

struct d3 {
    double x, y, z;
};

__device__ __forceinline__ d3 mk3(double x, double y, double z)
{
    d3 r;
    r.x = x; r.y = y; r.z = z;
    return r;
}
__device__ __forceinline__ d3 sub3(d3 a, d3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ double dot3(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross3(d3 a, d3 b)
{
    return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ d3 div3(d3 a, double s) { return mk3(a.x / s, a.y / s, a.z / s); }

// Philox4x64-10 (Salmon et al., SC'11): counter (i, src, stage, 0), key (seed, 0)
__device__ __forceinline__ void philox(uint64_t i, uint64_t src, uint64_t stage, uint64_t seed,
                                       uint64_t out[4])
{
    uint64_t c0 = i, c1 = src, c2 = stage, c3 = 0, k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

// sin and cos of 2 pi u: exact quarter-turn reduction, then the Taylor series
// of sin to x^17 and cos to x^18 on |x| <= pi/4, evaluated by Horner's rule
// in the same order as the CPU reference so that the results agree bitwise.
__device__ __forceinline__ void sincos_turn(double u, double &so, double &co)
{
    double n = __builtin_rint(4.0 * u);
    double r = u - 0.25 * n;
    double x = r * 6.283185307179586;
    double z = x * x;
    double ps = -1.0 / 355687428096000.0;
    ps = ps * z + 1.0 / 1307674368000.0;
    ps = ps * z - 1.0 / 6227020800.0;
    ps = ps * z + 1.0 / 39916800.0;
    ps = ps * z - 1.0 / 362880.0;
    ps = ps * z + 1.0 / 5040.0;
    ps = ps * z - 1.0 / 120.0;
    ps = ps * z + 1.0 / 6.0;
    double s = x - (x * z) * ps;
    double pc = 1.0 / 6402373705728000.0;
    pc = pc * z - 1.0 / 20922789888000.0;
    pc = pc * z + 1.0 / 87178291200.0;
    pc = pc * z - 1.0 / 479001600.0;
    pc = pc * z + 1.0 / 3628800.0;
    pc = pc * z - 1.0 / 40320.0;
    pc = pc * z + 1.0 / 720.0;
    pc = pc * z - 1.0 / 24.0;
    pc = pc * z + 0.5;
    double c = 1.0 - z * pc;
    int q = ((int)n) & 3;
    so = (q == 0) ? s : (q == 1) ? c : (q == 2) ? -s : -c;
    co = (q == 0) ? c : (q == 1) ? -s : (q == 2) ? -c : s;
}

#define RR_TMIN 1e-6

// Moller-Trumbore (1997) in FP64; closed triangle, t > RR_TMIN
__device__ __forceinline__ bool mt_hit(d3 o, d3 d, d3 v0, d3 v1, d3 v2, double &t_out)
{
    d3 e1 = sub3(v1, v0), e2 = sub3(v2, v0);
    d3 pv = cross3(d, e2);
    double det = dot3(e1, pv);
    if (det == 0.0) return false;
    double inv = 1.0 / det;
    d3 tv = sub3(o, v0);
    double u = dot3(tv, pv) * inv;
    if (!(u >= 0.0 && u <= 1.0)) return false;
    d3 qv = cross3(tv, e1);
    double v = dot3(d, qv) * inv;
    if (!(v >= 0.0 && u + v <= 1.0)) return false;
    double t = dot3(e2, qv) * inv;
    if (!(t > RR_TMIN)) return false;
    t_out = t;
    return true;
}

__device__ __forceinline__ float safe_inv(double d)
{
    float f = (float)d;
    if (fabsf(f) < 1e-30f) f = copysignf(1e-30f, f);
    return 1.0f / f;
}

// Work counters of the counting tracer (k_trace_count): BVH nodes fetched,
// leaf triangle records fetched, closest-hit queries.
struct TraceCount {
    unsigned nodes, tris, queries;
};

// Closest hit of the ray (o, d) over every triangle except `skip`: smallest
// t > RR_TMIN, lowest id on ties.  Returns the triangle id (-1: miss), its t
// and its position in the leaf-ordered triangle array.  CNT: also count the
// work into *cn.
template <bool CNT>
__device__ int closest_hit_t(const TraceArgs &A, d3 o, d3 d, int skip, double &tbest, int &lbest,
                             int *stk, TraceCount *cn)
{
    if (CNT) cn->queries++;
    int best = -1;
    tbest = __builtin_huge_val();
    lbest = -1;
    if (!A.has_bvh) return -1;
    const float ox = (float)o.x, oy = (float)o.y, oz = (float)o.z;
    const float ix = safe_inv(d.x), iy = safe_inv(d.y), iz = safe_inv(d.z);
    const float oix = ox * ix, oiy = oy * iy, oiz = oz * iz;
    float tmax = __builtin_huge_valf();
    int sp = 0;
    int ref = 0;
    while (true) {
        if (ref >= 0) {
            if (CNT) cn->nodes++;
            const float4 *N = A.nodes + 4 * (int64_t)ref;
            float4 n0 = N[0], n1 = N[1], n2 = N[2], n3 = N[3];
            float a0 = fmaf(n0.x, ix, -oix), a1 = fmaf(n0.w, ix, -oix);
            float b0 = fmaf(n0.y, iy, -oiy), b1 = fmaf(n1.x, iy, -oiy);
            float c0 = fmaf(n0.z, iz, -oiz), c1 = fmaf(n1.y, iz, -oiz);
            float tn0 = fmaxf(fmaxf(fminf(a0, a1), fminf(b0, b1)), fmaxf(fminf(c0, c1), 0.0f));
            float tf0 = fminf(fminf(fmaxf(a0, a1), fmaxf(b0, b1)), fminf(fmaxf(c0, c1), tmax));
            a0 = fmaf(n1.z, ix, -oix); a1 = fmaf(n2.y, ix, -oix);
            b0 = fmaf(n1.w, iy, -oiy); b1 = fmaf(n2.z, iy, -oiy);
            c0 = fmaf(n2.x, iz, -oiz); c1 = fmaf(n2.w, iz, -oiz);
            float tn1 = fmaxf(fmaxf(fminf(a0, a1), fminf(b0, b1)), fmaxf(fminf(c0, c1), 0.0f));
            float tf1 = fminf(fminf(fmaxf(a0, a1), fmaxf(b0, b1)), fminf(fmaxf(c0, c1), tmax));
            bool h0 = tn0 <= tf0, h1 = tn1 <= tf1;
            int r0 = __float_as_int(n3.x), r1 = __float_as_int(n3.y);
            if (h0 && h1) {
                bool first0 = tn0 <= tn1;
                int nearr = first0 ? r0 : r1, farr = first0 ? r1 : r0;
                if (sp < RR_STACK) {
                    stk[sp * RR_TRACE_BLOCK] = farr;
                    sp++;
                } else {
                    atomicOr(A.err_flag, 1);
                }
                ref = nearr;
                continue;
            }
            if (h0) { ref = r0; continue; }
            if (h1) { ref = r1; continue; }
        } else {
            int x = ~ref;
            int first = x >> 3, cnt = (x & 7) + 1;
            if (CNT) cn->tris += (unsigned)cnt;
            for (int k = 0; k < cnt; k++) {
                const float4 *T = A.ltris + 3 * (int64_t)(first + k);
                float4 t0 = T[0], t1 = T[1], t2 = T[2];
                int id = __float_as_int(t2.y);
                if (id == skip) continue;
                d3 v0 = mk3(t0.x, t0.y, t0.z), v1 = mk3(t0.w, t1.x, t1.y), v2 = mk3(t1.z, t1.w, t2.x);
                double th;
                if (mt_hit(o, d, v0, v1, v2, th) && (th < tbest || (th == tbest && id < best))) {
                    tbest = th;
                    best = id;
                    lbest = first + k;
                    float tf = (float)th;
                    if ((double)tf < th) tf = nextafterf(tf, __builtin_huge_valf());
                    tmax = tf;
                }
            }
        }
        if (sp == 0) break;
        sp--;
        ref = stk[sp * RR_TRACE_BLOCK];
    }
    return best;
}

__device__ __forceinline__ int closest_hit(const TraceArgs &A, d3 o, d3 d, int skip, double &tbest,
                                           int &lbest, int *stk)
{
    return closest_hit_t<false>(A, o, d, skip, tbest, lbest, stk, nullptr);
}

// Eqs. (1)-(3): n is the unit normal facing the incident direction d.
__device__ __forceinline__ d3 bounce_dir(d3 d, d3 n, double alpha, double u0, double u1)
{
    double dn = dot3(d, n);
    double s2 = 2.0 * dn;
    d3 m = mk3(d.x - s2 * n.x, d.y - s2 * n.y, d.z - s2 * n.z);
    double z = 1.0 - 2.0 * u0;
    double rho = sqrt(fmax(0.0, 1.0 - z * z));
    double sp, cp;
    sincos_turn(u1, sp, cp);
    d3 td = mk3(n.x + rho * cp, n.y + rho * sp, n.z + z);
    double tl = sqrt(dot3(td, td));
    td = (tl < 1e-12) ? n : div3(td, tl);
    double b = 1.0 - alpha;
    d3 tc = mk3(alpha * td.x + b * m.x, alpha * td.y + b * m.y, alpha * td.z + b * m.z);
    double cl = sqrt(dot3(tc, tc));
    return (cl < 1e-12) ? m : div3(tc, cl);
}

// first bin b with u < cdf[b + 1]
__device__ __forceinline__ int cdf_bin(const double *cdf, int nb, double u)
{
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (u < cdf[mid + 1]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

struct Rec {
    d3 P[RR_KMAX];
    int tri[RR_KMAX];
    int vid[RR_KMAX];
};

// one atomic per wavefront; every active lane must call this
__device__ __forceinline__ void append(const TraceArgs &A, bool rec, int32_t src, int K,
                                       int64_t v, int loc, const Rec &R, double L, double amp)
{
    unsigned long long m = __ballot(rec);
    if (!rec) return;
    int lane = __lane_id();
    int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long below = m & ((1ull << lane) - 1ull);
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(A.counter, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    int64_t slot = (int64_t)(base + (unsigned long long)__popcll(below));
    const PathSoA &T = A.tmp;
    if (slot >= T.cap) return;
    const int64_t cap = T.cap;
    T.src[slot] = src;
    T.K[slot] = K;
    T.ray[slot] = v;
    T.loc[slot] = loc;
#pragma unroll
    for (int q = 0; q < RR_KMAX; q++) {
        bool u = q < K;
        T.tri[q * cap + slot] = u ? R.tri[q] : -1;
        T.vid[q * cap + slot] = u ? R.vid[q] : -1;
        T.p[(3 * q + 0) * cap + slot] = u ? R.P[q].x : 0.0;
        T.p[(3 * q + 1) * cap + slot] = u ? R.P[q].y : 0.0;
        T.p[(3 * q + 2) * cap + slot] = u ? R.P[q].z : 0.0;
    }
    T.L[slot] = L;
    T.amp[slot] = amp;
}

// one launched ray g (source-major) through all of its bounces
template <bool CNT = false>
__device__ __forceinline__ void trace_from(const TraceArgs &A, d3 src, d3 dir, int64_t i, int64_t t, int64_t v,
                           double amp, int32_t srcid, int32_t *hrow, int *stk, int64_t target,
                           TraceCount *cn = nullptr);

// Per-triangle casting: ray i of a source aims at piece f = i / g^2 (a
// triangle, or part of one cut by the host's subdivision), at a point drawn
// uniformly in cell (k mod g, k / g), k = i mod g^2, of a g x g grid over the
// unit square and carried onto the piece by the area-preserving map
// (1 - sqrt u1) v0 + sqrt u1 (1 - u2) v1 + sqrt u1 u2 v2.  Weight
// p0 A |cos| / d^2 (A |cos| = |area normal . dir| / 2) over g^2 rays; only
// rays inside the field of view are traced, and they count only when the
// piece's triangle is their first hit.
template <bool CNT = false>
__device__ void trace_tri(const TraceArgs &A, int64_t g, int64_t t, int64_t i, int64_t v, d3 src,
                          int *stk, TraceCount *cn = nullptr)
{
    const int64_t gs = A.tri_g, gg = gs * gs;
    const int64_t f = i / gg, k = i - f * gg;
    int32_t *hrow = A.hits ? A.hits + g * (A.bmax + 1) : nullptr;
    uint64_t r[4];
    philox((uint64_t)i, (uint64_t)t, 0, A.seed, r);
    const double u1 = ((double)(k % gs) + u01(r[0])) / (double)gs;
    const double u2 = ((double)(k / gs) + u01(r[1])) / (double)gs;
    const double *T = A.pieces + 9 * f;
    const d3 v0 = mk3(T[0], T[1], T[2]), v1 = mk3(T[3], T[4], T[5]), v2 = mk3(T[6], T[7], T[8]);
    const double su = sqrt(u1);
    const double b0 = 1.0 - su, b1 = su * (1.0 - u2), b2 = su * u2;
    const d3 x = mk3(b0 * v0.x + b1 * v1.x + b2 * v2.x, b0 * v0.y + b1 * v1.y + b2 * v2.y,
                     b0 * v0.z + b1 * v1.z + b2 * v2.z);
    const d3 a = sub3(x, src);
    const double d2 = dot3(a, a);
    bool ok = d2 > 0.0;
    d3 d = div3(a, sqrt(d2));
    ok = ok && d.z >= A.slo && d.z <= A.shi;
    ok = ok && A.fov_c0 * d.y - A.fov_s0 * d.x >= 0.0 && A.fov_c1 * d.y - A.fov_s1 * d.x <= 0.0;
    const d3 na = cross3(sub3(v1, v0), sub3(v2, v0));
    const double w = (0.5 * fabs(dot3(na, d))) / (d2 * A.omega);
    ok = ok && w > 0.0;
    if (!ok) {
        if (hrow)
            for (int q = 0; q <= A.bmax; q++) hrow[q] = -1;
        A.counts[v] = 0;
        return;
    }
    trace_from<CNT>(A, src, d, i, t, v, w / (double)gg, A.shared ? -1 : (int32_t)t, hrow, stk,
                    A.piece_parent[f], cn);
}

// The first direction of ray i of source t as a point (fa, fs) of the unit
// square (azimuth fraction, sine of elevation fraction) and its weight:
// uniform, or a proposal bin drawn from the table and a point inside it.
__device__ __forceinline__ void primary_draw(const TraceArgs &A, int64_t t, int64_t i, double &fa,
                                             double &fs, double &w)
{
    uint64_t r[4];
    philox((uint64_t)i, (uint64_t)t, 0, A.seed, r);
    w = 1.0;
    if (A.sampler == RR_PROPOSAL) {
        int nb = A.n_az * A.n_el;
        int b = cdf_bin(A.cdf, nb, u01(r[0]));
        int ia = b % A.n_az, ie = b / A.n_az;
        fa = ((double)ia + u01(r[1])) / (double)A.n_az;
        fs = ((double)ie + u01(r[2])) / (double)A.n_el;
        double q = A.cdf[b + 1] - A.cdf[b];
        w = 1.0 / ((double)nb * q);
    } else {
        fa = u01(r[0]);
        fs = u01(r[1]);
    }
}

template <bool CNT = false>
__device__ void trace_ray(const TraceArgs &A, int64_t g, int *stk, TraceCount *cn = nullptr)
{
    int64_t t = g / A.n_per_src;
    int64_t i = g - t * A.n_per_src;
    int64_t v = A.vbase + t * A.n_virt_per_src + i;
    d3 src = A.shared ? mk3(A.oT[0], A.oT[1], A.oT[2])
                      : mk3(A.tx[3 * t], A.tx[3 * t + 1], A.tx[3 * t + 2]);
    if (A.sampler == RR_PER_TRIANGLE) {
        trace_tri<CNT>(A, g, t, i, v, src, stk, cn);
        return;
    }
    double fa, fs, w;
    primary_draw(A, t, i, fa, fs, w);
    double turn = A.at + fa * (A.bt - A.at);
    double sz = A.slo + fs * (A.shi - A.slo);
    double ce = sqrt(1.0 - sz * sz);
    double sa, ca;
    sincos_turn(turn, sa, ca);
    d3 dir = mk3(ce * ca, ce * sa, sz);
    const double amp = w / (double)A.n_per_src;
    const int32_t srcid = A.shared ? -1 : (int32_t)t;
    int32_t *hrow = A.hits ? A.hits + g * (A.bmax + 1) : nullptr;
    trace_from<CNT>(A, src, dir, i, t, v, amp, srcid, hrow, stk, -1, cn);
}

// Caller-supplied ray g: origin, direction (normalised here), amplitude and
// source from U; its bounce random numbers use the ray's index within its
// source's run of rays, so that the launch's own rays reproduce k_trace.
__device__ void trace_user(const TraceArgs &A, const UserRays &U, int64_t g, int *stk)
{
    const int32_t srcid = U.src[g];
    int64_t lo = 0, hi = g;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (U.src[mid] < srcid) lo = mid + 1; else hi = mid;
    }
    d3 o = mk3(U.orig[3 * g], U.orig[3 * g + 1], U.orig[3 * g + 2]);
    d3 d = mk3(U.dir[3 * g], U.dir[3 * g + 1], U.dir[3 * g + 2]);
    d = div3(d, sqrt(dot3(d, d)));
    int32_t *hrow = A.hits ? A.hits + g * (A.bmax + 1) : nullptr;
    trace_from(A, o, d, g - lo, srcid > 0 ? srcid : 0, A.vbase + g, U.amp[g], srcid, hrow, stk, -1);
}

// The bounces of one ray from o along the unit vector dir: closest hit,
// reception of every segment that follows a hit, the direction of Eqs. 1-3
// at each hit with the random numbers of counter (i, t, j + 1); paths carry
// source srcid, virtual ray v and amplitude amp.  target >= 0: the ray is
// dropped (hit row all -1, no paths) unless its first hit is that triangle.
template <bool CNT>
__device__ __forceinline__ void trace_from(const TraceArgs &A, d3 src, d3 dir, int64_t i, int64_t t, int64_t v,
                           double amp, int32_t srcid, int32_t *hrow, int *stk, int64_t target,
                           TraceCount *cn)
{
    Rec R;
#pragma unroll
    for (int q = 0; q < RR_KMAX; q++) {
        R.P[q] = mk3(0.0, 0.0, 0.0);
        R.tri[q] = -1;
        R.vid[q] = -1;
    }
    d3 o = src;
    double L = 0.0;
    int prev = -1;
    int n_emit = 0;
    int jlast = A.bmax;
    for (int j = 0; j <= A.bmax; j++) {
        double th;
        int lidx;
        int h = closest_hit_t<CNT>(A, o, dir, prev, th, lidx, stk, cn);
        if (j == 0 && target >= 0 && h != target) {
            // cast towards a triangle that is not its first hit: not counted
            if (hrow)
                for (int q = 0; q <= A.bmax; q++) hrow[q] = -1;
            A.counts[v] = 0;
            return;
        }
        if (hrow) hrow[j] = h;
        bool rec = false;
        if (j >= 1) {
            d3 w2 = sub3(mk3(A.oR[0], A.oR[1], A.oR[2]), o);
            double ts = dot3(w2, dir);
            if (ts > 0.0 && ts < th) {
                double cx = (o.x + ts * dir.x) - A.oR[0];
                double cy = (o.y + ts * dir.y) - A.oR[1];
                double cz = (o.z + ts * dir.z) - A.oR[2];
                rec = cx * cx + cy * cy + cz * cz <= A.r2;
            }
        }
        append(A, rec, srcid, j, v, n_emit, R, L, amp);
        n_emit += rec ? 1 : 0;
        if (h < 0 || j == A.bmax) {
            jlast = j;
            break;
        }
        d3 p = mk3(o.x + th * dir.x, o.y + th * dir.y, o.z + th * dir.z);
        L += th;
        const float4 *T = A.ltris + 3 * (int64_t)lidx;
        float4 t0 = T[0], t1 = T[1], t2 = T[2];
        d3 v0 = mk3(t0.x, t0.y, t0.z), v1 = mk3(t0.w, t1.x, t1.y), v2 = mk3(t1.z, t1.w, t2.x);
        d3 n = cross3(sub3(v1, v0), sub3(v2, v0));
        n = div3(n, sqrt(dot3(n, n)));
        if (dot3(n, dir) > 0.0) n = mk3(-n.x, -n.y, -n.z);
        int obj = __float_as_int(t2.z);
#pragma unroll
        for (int q = 0; q < RR_KMAX; q++) {
            if (q == j) {
                R.P[q] = p;
                R.tri[q] = h;
                R.vid[q] = obj;
            }
        }
        uint64_t rb[4];
        philox((uint64_t)i, (uint64_t)t, (uint64_t)(j + 1), A.seed, rb);
        dir = bounce_dir(dir, n, (double)t2.w, u01(rb[0]), u01(rb[1]));
        o = p;
        prev = h;
    }
    if (hrow)
        for (int j = jlast + 1; j <= A.bmax; j++) hrow[j] = -1;
    A.counts[v] = (uint8_t)n_emit;
}

// Point reflectors: one single-bounce path per (source, point) when both the
// source-to-point and point-to-receiver legs are unobstructed.
__device__ void trace_point(const TraceArgs &A, int64_t g, int *stk)
{
    int64_t t = g / A.npts, q = g - t * A.npts;
    int64_t v = A.vbase + t * A.n_virt_per_src + A.n_per_src + q;
    d3 src = A.shared ? mk3(A.oT[0], A.oT[1], A.oT[2])
                      : mk3(A.tx[3 * t], A.tx[3 * t + 1], A.tx[3 * t + 2]);
    d3 Q = mk3(A.pt_pos[3 * q], A.pt_pos[3 * q + 1], A.pt_pos[3 * q + 2]);
    d3 oR = mk3(A.oR[0], A.oR[1], A.oR[2]);
    d3 a = sub3(Q, src);
    double la = sqrt(dot3(a, a));
    d3 b = sub3(oR, Q);
    double lb = sqrt(dot3(b, b));
    double th;
    int lidx;
    closest_hit(A, src, div3(a, la), -1, th, lidx, stk);
    bool vis = !(th < la);
    closest_hit(A, Q, div3(b, lb), -1, th, lidx, stk);
    vis = vis && !(th < lb);
    Rec R;
#pragma unroll
    for (int k = 0; k < RR_KMAX; k++) {
        R.P[k] = mk3(0.0, 0.0, 0.0);
        R.tri[k] = -1;
        R.vid[k] = -1;
    }
    R.P[0] = Q;
    R.vid[0] = A.nobj + (int)q;
    append(A, vis, A.shared ? -1 : (int32_t)t, 1, v, 0, R, la, A.pt_ap[q] / (la * la * A.omega));
    A.counts[v] = vis ? 1 : 0;
}

// Tracing kernels ask for four wavefronts per SIMD (at most 128 VGPRs): the
// traversal is bound by the latency of dependent node fetches, and a fourth
// wavefront hides more of it than the ~20 registers the compiler then keeps
// in scratch memory cost (street, 1e7 rays: 4.38 against 4.79 ms with three
// wavefronts and no spills; five wavefronts spill ~145 registers and lose).
#define RR_TRACE_WAVES 4

// lane g traces ray order[g] when a coherent order is given, else ray g
__global__ __launch_bounds__(RR_TRACE_BLOCK, RR_TRACE_WAVES) void k_trace(TraceArgs A, int64_t n_traced)
{
    __shared__ int lds_stack[RR_STACK * RR_TRACE_BLOCK];
    const int64_t g = (int64_t)blockIdx.x * RR_TRACE_BLOCK + threadIdx.x;
    if (g < n_traced) trace_ray(A, A.order ? (int64_t)A.order[g] : g, lds_stack + threadIdx.x);
}

// k_trace with work counters: the same rays, hits and paths, plus the sums
// over all rays of BVH nodes fetched, leaf triangle records fetched and
// closest-hit queries (stats[0..2], integer atomics: exact, order-free)
__global__ __launch_bounds__(RR_TRACE_BLOCK) void k_trace_count(TraceArgs A, int64_t n_traced,
                                                                unsigned long long *stats)
{
    __shared__ int lds_stack[RR_STACK * RR_TRACE_BLOCK];
    const int64_t g = (int64_t)blockIdx.x * RR_TRACE_BLOCK + threadIdx.x;
    TraceCount cn = {0u, 0u, 0u};
    if (g < n_traced) trace_ray<true>(A, A.order ? (int64_t)A.order[g] : g, lds_stack + threadIdx.x, &cn);
    unsigned long long a = cn.nodes, b = cn.tris, q = cn.queries;
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        q += __shfl_xor(q, off);
    }
    if (__lane_id() == 0) {
        atomicAdd(stats + 0, a);
        atomicAdd(stats + 1, b);
        atomicAdd(stats + 2, q);
    }
}

__global__ __launch_bounds__(RR_TRACE_BLOCK, RR_TRACE_WAVES) void k_trace_user(TraceArgs A, UserRays U)
{
    __shared__ int lds_stack[RR_STACK * RR_TRACE_BLOCK];
    const int64_t g = (int64_t)blockIdx.x * RR_TRACE_BLOCK + threadIdx.x;
    if (g < U.n) trace_user(A, U, g, lds_stack + threadIdx.x);
}

// flag = 1 if a source is out of range (-1 only, for a shared launch) or
// below its predecessor, or a vector is non-finite or zero
__global__ void k_check_user(UserRays U, int shared, int ntx, int *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= U.n) return;
    const int32_t t = U.src[i];
    bool bad = shared ? t != -1 : (t < 0 || t >= ntx || (i > 0 && t < U.src[i - 1]));
    double ss = 0.0;
    for (int a = 0; a < 3; a++) {
        bad = bad || !isfinite(U.orig[3 * i + a]) || !isfinite(U.dir[3 * i + a]);
        ss += fabs(U.dir[3 * i + a]);
    }
    bad = bad || !isfinite(U.amp[i]) || ss == 0.0;
    if (bad) *flag = 1;
}

__global__ __launch_bounds__(RR_TRACE_BLOCK) void k_points(TraceArgs A)
{
    __shared__ int lds_stack[RR_STACK * RR_TRACE_BLOCK];
    const int64_t g = (int64_t)blockIdx.x * RR_TRACE_BLOCK + threadIdx.x;
    if (g < A.n_src * (int64_t)A.npts) trace_point(A, g, lds_stack + threadIdx.x);
}

// Batched, persistent: the launched rays and the point reflectors of every
// scene are cut into chunks of one workgroup; workgroups pull chunk indices
// from a device counter until the queue is empty.  chunk_start[s] is the
// first chunk of scene s (S + 1 entries); scene s's rays come before its
// point reflectors.
__global__ __launch_bounds__(RR_TRACE_BLOCK, RR_TRACE_WAVES) void k_batch_trace(const TraceArgs *scenes,
                                                                const int64_t *chunk_start, int S,
                                                                unsigned long long *work)
{
    __shared__ int lds_stack[RR_STACK * RR_TRACE_BLOCK];
    __shared__ long long s_chunk;
    const int64_t n_chunks = chunk_start[S];
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_chunk = (long long)atomicAdd(work, 1ull);
        __syncthreads();
        const int64_t ch = s_chunk;
        if (ch >= n_chunks) break;
        int lo = 0, hi = S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (chunk_start[mid] <= ch) lo = mid; else hi = mid - 1;
        }
        const TraceArgs &A = scenes[lo];
        const int64_t c = ch - chunk_start[lo];
        const int64_t n_traced = A.n_src * A.n_per_src;
        const int64_t ray_chunks = (n_traced + RR_TRACE_BLOCK - 1) / RR_TRACE_BLOCK;
        if (c < ray_chunks) {
            const int64_t g = c * RR_TRACE_BLOCK + threadIdx.x;
            if (g < n_traced) trace_ray(A, g, lds_stack + threadIdx.x);
        } else {
            const int64_t g = (c - ray_chunks) * RR_TRACE_BLOCK + threadIdx.x;
            if (g < A.n_src * (int64_t)A.npts) trace_point(A, g, lds_stack + threadIdx.x);
        }
    }
}

// Scene code of the learned proposal: 16 azimuth sectors x 8 probe rays at
// elevation 0 from the Tx phase centre (sector k ray i at azimuth fraction
// (8 k + i + 1/2) / 128 of the field of view); code[k] = mean over the
// sector's rays of exp(-t / 10 m) for hits on objects other than object 0.
__global__ __launch_bounds__(RR_TRACE_BLOCK) void k_probe(TraceArgs A, float *code)
{
    __shared__ int lds_stack[RR_STACK * RR_TRACE_BLOCK];
    __shared__ double vals[128];
    int *stk = lds_stack + threadIdx.x;
    const int t = threadIdx.x;
    const int k = t >> 3, i = t & 7;
    const double fa = ((double)(8 * k + i) + 0.5) / 128.0;
    const double turn = A.at + fa * (A.bt - A.at);
    double sa, ca;
    sincos_turn(turn, sa, ca);
    double th;
    int lidx;
    const int h = closest_hit(A, mk3(A.oT[0], A.oT[1], A.oT[2]), mk3(ca, sa, 0.0), -1, th, lidx, stk);
    double val = 0.0;
    if (h >= 0) {
        const int obj = __float_as_int(A.ltris[3 * (int64_t)lidx + 2].z);
        if (obj != 0) val = exp(-th / 10.0);
    }
    vals[t] = val;
    __syncthreads();
    if (i == 0) {
        double acc = 0.0;
        for (int j = 0; j < 8; j++) acc += vals[8 * k + j];
        code[k] = (float)(acc / 8.0);
    }
}

// Training target of the proposal from a uniform trace: per direction bin the
// sum over its rays of (returned power = number of received paths, since
// w = 1) + 0.1 x (first segment hit an object other than object 0).
// Every ray adds a whole number of tenths, so the bins count tenths in 32-bit
// integers (the sum does not depend on the order of the atomic adds) and
// k_hist_finish turns the counts into values in place.
__global__ void k_hist(TraceArgs A, int64_t n_traced, const int32_t *hits, const int32_t *tri_obj,
                       int n_az, int n_el, unsigned *H)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_traced) return;
    const int64_t t = g / A.n_per_src;
    const int64_t i = g - t * A.n_per_src;
    const int64_t v = t * A.n_virt_per_src + i;
    uint64_t r[4];
    philox((uint64_t)i, (uint64_t)t, 0, A.seed, r);
    int ia = (int)(u01(r[0]) * n_az), ie = (int)(u01(r[1]) * n_el);
    ia = min(ia, n_az - 1);
    ie = min(ie, n_el - 1);
    const int h0 = hits[g * (A.bmax + 1)];
    const unsigned tenths = 10u * (unsigned)A.counts[v] + ((h0 >= 0 && tri_obj[h0] != 0) ? 1u : 0u);
    if (tenths != 0u) atomicAdd(&H[ie * n_az + ia], tenths);
}

__global__ void k_hist_finish(float *H, int nb)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const unsigned u = reinterpret_cast<const unsigned *>(H)[b];
    H[b] = (float)((double)u / 10.0);
}

// ---------------------------------------------------------------------------
// exclusive scan of uint8 counts -> uint32 offsets (three passes)
// ---------------------------------------------------------------------------
#define SCAN_T 256
#define SCAN_PER 16
#define SCAN_TILE (SCAN_T * SCAN_PER)

__device__ __forceinline__ uint32_t load16_sum(const uint8_t *c, int64_t base, int64_t n, uint32_t v[16])
{
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        int64_t idx = base + k;
        v[k] = idx < n ? c[idx] : 0u;
        s += v[k];
    }
    return s;
}

__device__ uint32_t block_excl_scan(uint32_t x, uint32_t *sh, uint32_t &total)
{
    // Hillis-Steele over the block in LDS (SCAN_T threads)
    int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        uint32_t y = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    uint32_t incl = sh[t];
    total = sh[SCAN_T - 1];
    __syncthreads();
    return incl - x;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const uint8_t *c, int64_t n, uint32_t *bsums)
{
    __shared__ uint32_t sh[SCAN_T];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    uint32_t v[16];
    uint32_t s = load16_sum(c, base, n, v);
    uint32_t tot;
    block_excl_scan(s, sh, tot);
    if (threadIdx.x == 0) bsums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_top(uint32_t *bsums, int64_t nb,
                                                     unsigned long long *total)
{
    __shared__ uint32_t sh[SCAN_T];
    unsigned long long carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += SCAN_T) {
        int64_t b = b0 + threadIdx.x;
        uint32_t x = b < nb ? bsums[b] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(x, sh, tot);
        if (b < nb) bsums[b] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const uint8_t *c, int64_t n,
                                                       const uint32_t *boffs, uint32_t *offs)
{
    __shared__ uint32_t sh[SCAN_T];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER;
    uint32_t v[16];
    uint32_t s = load16_sum(c, base, n, v);
    uint32_t tot;
    uint32_t run = boffs[blockIdx.x] + block_excl_scan(s, sh, tot);
#pragma unroll
    for (int k = 0; k < 16; k++) {
        int64_t idx = base + k;
        if (idx < n) offs[idx] = run;
        run += v[k];
    }
}

__global__ void k_scatter(PathSoA tmp, const unsigned long long *counter, int64_t tmp_cap,
                          const uint32_t *offs, PathSoA dst, int64_t keep)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = (int64_t)*counter;
    if (n > tmp_cap) n = tmp_cap;
    if (s >= n) return;
    int64_t d = (int64_t)offs[tmp.ray[s]] + tmp.loc[s];
    if (d >= keep) return;
    const int64_t sc = tmp.cap, dc = dst.cap;
    dst.src[d] = tmp.src[s];
    dst.K[d] = tmp.K[s];
    dst.ray[d] = tmp.ray[s];
#pragma unroll
    for (int q = 0; q < RR_KMAX; q++) {
        dst.tri[q * dc + d] = tmp.tri[q * sc + s];
        dst.vid[q * dc + d] = tmp.vid[q * sc + s];
    }
#pragma unroll
    for (int q = 0; q < 3 * RR_KMAX; q++) dst.p[q * dc + d] = tmp.p[q * sc + s];
    dst.L[d] = tmp.L[s];
    dst.amp[d] = tmp.amp[s];
}

// Material mix of every leaf triangle (word 11 of its 12-word record): the
// per-face value indexed by the triangle's upload index (word 9) when given,
// else its object's (object index in word 10).  No BVH rebuild needed.
__global__ void k_set_alpha(float *ltris, int64_t n, const float *tri_alpha, const float *obj_alpha)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float *T = ltris + 12 * k;
    const int id = __float_as_int(T[9]), obj = __float_as_int(T[10]);
    T[11] = tri_alpha ? tri_alpha[id] : obj_alpha[obj];
}

// Coherent ray order.  The rays of one source are sorted by the cell of their
// first direction: 2^b x 2^b cells of the unit square that direction is drawn
// from, in Morton order, so that a wavefront's rays leave their source
// together and walk the same BVH nodes.  A counting sort over chunks of one
// source's rays (four rays a cell per chunk): a workgroup counts its chunk's
// cells in LDS and adds the non-zero counts to the global ones; after the
// scan it reserves each cell's range with one atomic and places its rays
// inside it (the order inside a cell is whatever the atomics give).  Nothing
// a ray computes depends on the lane that takes it: its random numbers follow
// its index, and its hit row, count and path records are written there.
__device__ __forceinline__ unsigned spread_bits(unsigned x)
{
    x &= 0xffu;
    x = (x | (x << 4)) & 0x0f0fu;
    x = (x | (x << 2)) & 0x3333u;
    x = (x | (x << 1)) & 0x5555u;
    return x;
}

// cell of ray i of source t within its source's 4^bits cells
__device__ __forceinline__ unsigned ray_cell(const TraceArgs &A, int64_t t, int64_t i, int bits)
{
    double fa, fs, w;
    primary_draw(A, t, i, fa, fs, w);
    const int n = 1 << bits;
    const unsigned ca = (unsigned)min((int)(fa * n), n - 1);
    const unsigned cs = (unsigned)min((int)(fs * n), n - 1);
    return spread_bits(ca) | (spread_bits(cs) << 1);
}

// workgroup blockIdx.x: chunk c of source t, rays [lo, hi)
__device__ __forceinline__ void order_chunk(const TraceArgs &A, int64_t chunk, int64_t &t,
                                            int64_t &lo, int64_t &hi)
{
    const int64_t per = (A.n_per_src + chunk - 1) / chunk;
    t = blockIdx.x / per;
    lo = (int64_t)(blockIdx.x - t * per) * chunk;
    hi = min(lo + chunk, A.n_per_src);
}

#define RR_ORDER_T 512

__global__ __launch_bounds__(RR_ORDER_T) void k_order_count(TraceArgs A, int bits, int64_t chunk,
                                                            uint16_t *cells, unsigned *cnt)
{
    extern __shared__ unsigned hist[];
    const int nb = 1 << (2 * bits);
    int64_t t, lo, hi;
    order_chunk(A, chunk, t, lo, hi);
    for (int b = threadIdx.x; b < nb; b += RR_ORDER_T) hist[b] = 0u;
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += RR_ORDER_T) {
        const unsigned c = ray_cell(A, t, i, bits);
        cells[t * A.n_per_src + i] = (uint16_t)c;
        atomicAdd(&hist[c], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += RR_ORDER_T)
        if (hist[b]) atomicAdd(cnt + t * nb + b, hist[b]);
}

// exclusive scan in place of source blockIdx.x's nb cell counts, offset by
// the source's first position (every source has n_per_src rays): one
// workgroup of 1024 threads a source, each over a contiguous run
__global__ __launch_bounds__(1024) void k_order_scan(unsigned *cells, int64_t nb, int64_t n_per_src)
{
    __shared__ unsigned part[1024];
    unsigned *c = cells + (int64_t)blockIdx.x * nb;
    const int tid = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t lo = min(nb, (int64_t)tid * per), hi = min(nb, lo + per);
    unsigned s = 0;
    for (int64_t k = lo; k < hi; k++) s += c[k];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned v = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    unsigned run = (unsigned)((int64_t)blockIdx.x * n_per_src) + (tid ? part[tid - 1] : 0u);
    for (int64_t k = lo; k < hi; k++) {
        const unsigned x = c[k];
        c[k] = run;
        run += x;
    }
}

__global__ __launch_bounds__(RR_ORDER_T) void k_order_place(TraceArgs A, int bits, int64_t chunk,
                                                            const uint16_t *cells, unsigned *cur,
                                                            int32_t *order)
{
    extern __shared__ unsigned hist[];
    const int nb = 1 << (2 * bits);
    int64_t t, lo, hi;
    order_chunk(A, chunk, t, lo, hi);
    const uint16_t *cl = cells + t * A.n_per_src;
    for (int b = threadIdx.x; b < nb; b += RR_ORDER_T) hist[b] = 0u;
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += RR_ORDER_T) atomicAdd(&hist[cl[i]], 1u);
    __syncthreads();
    // this chunk's range of every cell it holds
    for (int b = threadIdx.x; b < nb; b += RR_ORDER_T) {
        const unsigned v = hist[b];
        hist[b] = v ? atomicAdd(cur + t * nb + b, v) : 0u;
    }
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += RR_ORDER_T)
        order[atomicAdd(&hist[cl[i]], 1u)] = (int32_t)(t * A.n_per_src + i);
}

}  // namespace

hipError_t launch_set_alpha(float4 *ltris, int64_t n_tris, const float *tri_alpha,
                            const float *obj_alpha, hipStream_t s)
{
    if (n_tris <= 0) return hipSuccess;
    if (!tri_alpha && !obj_alpha) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((n_tris + 255) / 256);
    hipLaunchKernelGGL(k_set_alpha, dim3(blocks), dim3(256), 0, s, reinterpret_cast<float *>(ltris),
                       n_tris, tri_alpha, obj_alpha);
    return hipGetLastError();
}

// cells per source: 4^b with about 128-512 rays a cell (a sweep of cell sizes
// found ~200 best for 8e5 and 4e6 rays per source), at most 128 x 128 (the
// LDS counts of a workgroup, 64 KiB; cell numbers fit 16 bits)
#define RR_ORDER_MAXBITS 7
#define RR_ORDER_CELL 128
static_assert(RR_ORDER_MAXBITS <= 7, "cell counts must fit 64 KiB of LDS");
int trace_order_bits(int64_t n_per_src)
{
    int bits = 0;
    while (bits < RR_ORDER_MAXBITS && (n_per_src >> (2 * bits + 2)) >= RR_ORDER_CELL) bits++;
    return bits;
}

hipError_t launch_trace_order(const TraceArgs &a, int64_t n_traced, int bits, unsigned *cells,
                              uint16_t *ray_cells, int32_t *order, hipStream_t s)
{
    if (n_traced <= 0) return hipSuccess;
    if (bits > RR_ORDER_MAXBITS || n_traced != a.n_src * a.n_per_src) return hipErrorInvalidValue;
    const int64_t nb = (int64_t)1 << (2 * bits), nk = a.n_src * nb;
    hipError_t e = hipMemsetAsync(cells, 0, (size_t)nk * 4, s);
    if (e != hipSuccess) return e;
    const int64_t chunk = 4 * nb;
    const int64_t blocks = a.n_src * ((a.n_per_src + chunk - 1) / chunk);
    const size_t lds = (size_t)nb * 4;
    hipLaunchKernelGGL(k_order_count, dim3((unsigned)blocks), dim3(RR_ORDER_T), lds, s, a, bits, chunk,
                       ray_cells, cells);
    hipLaunchKernelGGL(k_order_scan, dim3((unsigned)a.n_src), dim3(1024), 0, s, cells, nb, a.n_per_src);
    hipLaunchKernelGGL(k_order_place, dim3((unsigned)blocks), dim3(RR_ORDER_T), lds, s, a, bits, chunk,
                       ray_cells, cells, order);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs &a, int64_t n_traced, hipStream_t s)
{
    if (n_traced <= 0) return hipSuccess;
    int64_t blocks = (n_traced + RR_TRACE_BLOCK - 1) / RR_TRACE_BLOCK;
    hipLaunchKernelGGL(k_trace, dim3((unsigned)blocks), dim3(RR_TRACE_BLOCK), 0, s, a, n_traced);
    return hipGetLastError();
}

hipError_t launch_trace_count(const TraceArgs &a, int64_t n_traced, unsigned long long *stats,
                              hipStream_t s)
{
    if (n_traced <= 0) return hipSuccess;
    int64_t blocks = (n_traced + RR_TRACE_BLOCK - 1) / RR_TRACE_BLOCK;
    hipLaunchKernelGGL(k_trace_count, dim3((unsigned)blocks), dim3(RR_TRACE_BLOCK), 0, s, a, n_traced,
                       stats);
    return hipGetLastError();
}

hipError_t launch_trace_user(const TraceArgs &a, const UserRays &u, hipStream_t s)
{
    if (u.n <= 0) return hipSuccess;
    int64_t blocks = (u.n + RR_TRACE_BLOCK - 1) / RR_TRACE_BLOCK;
    hipLaunchKernelGGL(k_trace_user, dim3((unsigned)blocks), dim3(RR_TRACE_BLOCK), 0, s, a, u);
    return hipGetLastError();
}

hipError_t launch_check_user(const UserRays &u, int shared, int ntx, int *flag, hipStream_t s)
{
    if (u.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_user, dim3((unsigned)((u.n + 255) / 256)), dim3(256), 0, s, u,
                       shared, ntx, flag);
    return hipGetLastError();
}

hipError_t launch_points(const TraceArgs &a, hipStream_t s)
{
    int64_t n = a.n_src * (int64_t)a.npts;
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + RR_TRACE_BLOCK - 1) / RR_TRACE_BLOCK;
    hipLaunchKernelGGL(k_points, dim3((unsigned)blocks), dim3(RR_TRACE_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_trace(const TraceArgs *scenes, const int64_t *chunk_start, int S,
                              int64_t n_chunks, unsigned long long *work, hipStream_t s)
{
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t grid = std::min<int64_t>(n_chunks, (int64_t)cus * 16);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_trace, dim3((unsigned)grid), dim3(RR_TRACE_BLOCK), 0, s, scenes,
                       chunk_start, S, work);
    return hipGetLastError();
}

hipError_t launch_probe(const TraceArgs &a, float *code, hipStream_t s)
{
    hipLaunchKernelGGL(k_probe, dim3(1), dim3(RR_TRACE_BLOCK), 0, s, a, code);
    return hipGetLastError();
}

hipError_t launch_hist(const TraceArgs &a, int64_t n_traced, const int32_t *hits,
                       const int32_t *tri_obj, int n_az, int n_el, float *H, hipStream_t s)
{
    if (n_traced <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_hist, dim3((unsigned)((n_traced + 255) / 256)), dim3(256), 0, s, a,
                       n_traced, hits, tri_obj, n_az, n_el, reinterpret_cast<unsigned *>(H));
    hipLaunchKernelGGL(k_hist_finish, dim3((unsigned)((n_az * n_el + 255) / 256)), dim3(256), 0, s, H,
                       n_az * n_el);
    return hipGetLastError();
}

int64_t scan_u8_blocks(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }

hipError_t launch_scan_u8(const uint8_t *counts, int64_t n, uint32_t *offsets, uint32_t *bsums,
                          int64_t nb_cap, unsigned long long *total, hipStream_t s)
{
    int64_t nb = scan_u8_blocks(n);
    if (nb > nb_cap) return hipErrorInvalidValue;
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, s, bsums, (int64_t)0, total);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, s, counts, n, bsums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, s, bsums, nb, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_T), 0, s, counts, n, bsums,
                       offsets);
    return hipGetLastError();
}

hipError_t launch_scatter(const PathSoA &tmp, const unsigned long long *counter, int64_t tmp_cap,
                          const uint32_t *offsets, const PathSoA &dst, int64_t keep,
                          hipStream_t s)
{
    if (tmp_cap <= 0 || keep <= 0) return hipSuccess;
    int64_t blocks = (tmp_cap + 255) / 256;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, s, tmp, counter, tmp_cap,
                       offsets, dst, keep);
    return hipGetLastError();
}
