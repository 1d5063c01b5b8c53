/*
 * oracle.c -- plain, slow, single-threaded FP64 reference of the radar
 * ray-tracing hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it is used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark.  It shares no code with the GPU path.
 *
 * What it computes (Braeunig et al., "A Realistic Radar Ray Tracing Simulator
 * for Hand Pose Imaging", Section III):
 *   - rays leave every transmitter (Sec. III-A, last paragraph) and are
 *     intersected with a triangle mesh (Sec. III);
 *   - at each hit the outgoing direction mixes a Lambertian lobe n + r
 *     (Eq. 1) and the mirror direction (Eq. 2, read as the law of reflection
 *     d - 2 (d.n) n) with the weight alpha (Eq. 3);
 *   - rays that are received accumulate their total path length d
 *     (Sec. III-B), and the baseband is the coherent sum of exp(-j 2 pi f d / c)
 *     over received paths (Eq. 4), with the stepped frequency replaced by the
 *     FMCW instantaneous frequency f_k = f0 + B k / K of fast-time sample k.
 * The paper leaves ray generation and reception to its reference simulator;
 * the readings used here (uniform launch in solid angle, an array-level
 * reception sphere, two-sided surfaces, FP64 Moller-Trumbore with
 * lowest-id tie break, Philox4x64-10 random numbers, point reflectors,
 * constant object velocities with stop-and-go chirps) are listed in the
 * design notes and are the same readings the GPU path implements.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, no
 * fast-math: every double operation is a single IEEE operation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* public structs (mirrored by ctypes in oracle/__init__.py)                */
/* ------------------------------------------------------------------------ */

typedef struct {
    const float *verts;      /* [nv][3] */
    int64_t nv;
    const int32_t *tris;     /* [nt][3] */
    const int32_t *tri_obj;  /* [nt] */
    int64_t nt;
    const float *obj_alpha;  /* [nobj] */
    const double *obj_vel;   /* [nobj][3] */
    int32_t nobj;
    const double *pt_pos;    /* [npts][3] */
    const double *pt_vel;    /* [npts][3] */
    const double *pt_ap;     /* [npts] aperture, m^2 */
    int32_t npts;
    const float *tri_alpha;  /* [nt] per-triangle alpha, or NULL: the object's */
} orc_scene;

typedef struct {
    const double *tx; int32_t ntx;
    const double *rx; int32_t nrx;
    double rx_radius;
    int32_t shared;          /* 0: rays from every Tx; 1: rays from the Tx phase centre */
} orc_array;

typedef struct {
    double f0, bandwidth, t_chirp, t_rep;
    int32_t n_samples, n_chirps;
} orc_chirp;

typedef struct {
    int64_t n_rays;
    int32_t max_bounces;
    uint64_t seed;
    double az_min, az_max, el_min, el_max;
    /* importance proposal over an n_az x n_el grid of equal solid angle bins
     * (bin b = ie * n_az + ia); cdf has n_az*n_el + 1 entries, cdf[0] = 0,
     * cdf[nb] = 1.  cdf == NULL selects uniform sampling. */
    const double *cdf;
    int32_t n_az, n_el;
    /* per-triangle casting when tri_g > 0: tri_g^2 rays towards every
     * triangle from every source (n_rays is then unused); with
     * tri_omega_max > 0 each triangle is first cut into pieces (below) */
    int32_t tri_g;
    double tri_omega_max;    /* sr; 0: no subdivision */
    int32_t tri_depth_max;   /* at most 4^depth pieces per triangle */
} orc_trace_params;

#define ORC_KMAX 8
typedef struct {
    int32_t src;             /* Tx index, -1 for a shared launch */
    int32_t K;               /* number of hit points (bounce order) */
    int64_t ray;             /* virtual ray id */
    int32_t tri[ORC_KMAX];   /* triangle of each hit, -1 for a point reflector */
    int32_t vid[ORC_KMAX];   /* velocity id: object id, or nobj + point id */
    double p[ORC_KMAX][3];   /* hit points at t = 0 */
    double L;                /* source -> p_K length at t = 0 */
    double amp;              /* amplitude a_p */
} orc_path;

#define ORC_TMIN 1e-6

/* ------------------------------------------------------------------------ */
/* vectors                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct { double x, y, z; } vec3;

static vec3 mk(double x, double y, double z) { vec3 r = {x, y, z}; return r; }
static vec3 vsub(vec3 a, vec3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static double vdot(vec3 a, vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static vec3 vcross(vec3 a, vec3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double vlen(vec3 a) { return sqrt(vdot(a, a)); }
static vec3 vdiv(vec3 a, double s) { return mk(a.x / s, a.y / s, a.z / s); }
static vec3 vload3d(const double *p) { return mk(p[0], p[1], p[2]); }
static vec3 vload3f(const float *p) { return mk((double)p[0], (double)p[1], (double)p[2]); }

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)                         */
/* ------------------------------------------------------------------------ */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    __uint128_t p = (__uint128_t)a * (__uint128_t)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ULL, c0, &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ULL, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform in [0, 1) */
static double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

static void draw(uint64_t seed, uint64_t i, uint64_t src, uint64_t stage, double u[4])
{
    uint64_t ctr[4] = {i, src, stage, 0}, key[2] = {seed, 0}, o[4];
    orc_philox4x64(ctr, key, o);
    for (int k = 0; k < 4; k++) u[k] = u01(o[k]);
}

/* ------------------------------------------------------------------------ */
/* sin and cos of 2 pi u (u in turns): exact quarter-turn reduction followed
 * by the Taylor series of sin to x^17 and cos to x^18 on |x| <= pi/4
 * (truncation < 1e-19).  The GPU tracer evaluates the same steps so that
 * ray directions agree bit for bit; the result is checked against libm.    */
/* ------------------------------------------------------------------------ */

void orc_sincos_turn(double u, double *s_out, double *c_out)
{
    double n = rint(4.0 * u);
    double r = u - 0.25 * n;                 /* exact, |r| <= 1/8 */
    double x = r * 6.283185307179586;        /* 2 pi */
    double z = x * x;
    double ps = -1.0 / 355687428096000.0;    /* -1/17! */
    ps = ps * z + 1.0 / 1307674368000.0;     /*  1/15! */
    ps = ps * z - 1.0 / 6227020800.0;        /* -1/13! */
    ps = ps * z + 1.0 / 39916800.0;          /*  1/11! */
    ps = ps * z - 1.0 / 362880.0;            /* -1/9!  */
    ps = ps * z + 1.0 / 5040.0;              /*  1/7!  */
    ps = ps * z - 1.0 / 120.0;               /* -1/5!  */
    ps = ps * z + 1.0 / 6.0;                 /*  1/3!  */
    /* ps = 1/3! - z/5! + z^2/7! - ..., so x - x z ps is the sine series */
    double s = x - (x * z) * ps;
    double pc = 1.0 / 6402373705728000.0;    /*  1/18! */
    pc = pc * z - 1.0 / 20922789888000.0;    /* -1/16! */
    pc = pc * z + 1.0 / 87178291200.0;       /*  1/14! */
    pc = pc * z - 1.0 / 479001600.0;         /* -1/12! */
    pc = pc * z + 1.0 / 3628800.0;           /*  1/10! */
    pc = pc * z - 1.0 / 40320.0;             /* -1/8!  */
    pc = pc * z + 1.0 / 720.0;               /*  1/6!  */
    pc = pc * z - 1.0 / 24.0;                /* -1/4!  */
    pc = pc * z + 0.5;                       /*  1/2!  */
    double c = 1.0 - z * pc;                 /* pc = 1/2! - z/4! + ... */
    long q = ((long)n) & 3;
    switch (q) {
    case 0: *s_out = s; *c_out = c; break;
    case 1: *s_out = c; *c_out = -s; break;
    case 2: *s_out = -s; *c_out = -c; break;
    default: *s_out = -c; *c_out = s; break;
    }
}

/* ------------------------------------------------------------------------ */
/* ray-triangle intersection: Moller & Trumbore (1997) in FP64               */
/* ------------------------------------------------------------------------ */

static int mt_hit(vec3 o, vec3 d, vec3 v0, vec3 v1, vec3 v2, double *t_out)
{
    vec3 e1 = vsub(v1, v0), e2 = vsub(v2, v0);
    vec3 pv = vcross(d, e2);
    double det = vdot(e1, pv);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    vec3 tv = vsub(o, v0);
    double u = vdot(tv, pv) * inv;
    if (!(u >= 0.0 && u <= 1.0)) return 0;
    vec3 qv = vcross(tv, e1);
    double v = vdot(d, qv) * inv;
    if (!(v >= 0.0 && u + v <= 1.0)) return 0;
    double t = vdot(e2, qv) * inv;
    if (!(t > ORC_TMIN)) return 0;
    *t_out = t;
    return 1;
}

static void tri_verts(const orc_scene *sc, int64_t i, vec3 *v0, vec3 *v1, vec3 *v2)
{
    const int32_t *t = sc->tris + 3 * i;
    *v0 = vload3f(sc->verts + 3 * (int64_t)t[0]);
    *v1 = vload3f(sc->verts + 3 * (int64_t)t[1]);
    *v2 = vload3f(sc->verts + 3 * (int64_t)t[2]);
}

/* closest hit over every triangle: smallest t > TMIN, excluding `skip`;
 * equal t keeps the lowest triangle id. */
static int64_t closest_brute(const orc_scene *sc, vec3 o, vec3 d, int64_t skip, double *t_best)
{
    int64_t best = -1;
    double tb = INFINITY;
    for (int64_t i = 0; i < sc->nt; i++) {
        if (i == skip) continue;
        vec3 v0, v1, v2;
        double t;
        tri_verts(sc, i, &v0, &v1, &v2);
        if (mt_hit(o, d, v0, v1, v2, &t) && t < tb) { tb = t; best = i; }
    }
    *t_best = tb;
    return best;
}

/* ------------------------------------------------------------------------ */
/* a simple median-split BVH (object median on the widest centroid axis),    */
/* used only to make the oracle finish on large scenes; it must give the     */
/* same answer as closest_brute (checked by the tests).                      */
/* ------------------------------------------------------------------------ */

typedef struct { double lo[3], hi[3]; int64_t left, right, first, count; } onode;

typedef struct {
    onode *nodes; int64_t n_nodes;
    int64_t *idx;
    double *cent;            /* [nt][3] */
} obvh;

static obvh g_bvh;
static const orc_scene *g_bvh_scene;
static int g_sort_axis;

static int cmp_cent(const void *a, const void *b)
{
    double ca = g_bvh.cent[3 * *(const int64_t *)a + g_sort_axis];
    double cb = g_bvh.cent[3 * *(const int64_t *)b + g_sort_axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    return ia < ib ? -1 : (ia > ib);
}

static int64_t bvh_build_rec(const orc_scene *sc, int64_t first, int64_t count)
{
    int64_t me = g_bvh.n_nodes++;
    onode *nd = &g_bvh.nodes[me];
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int a = 0; a < 3; a++) { nd->lo[a] = INFINITY; nd->hi[a] = -INFINITY; }
    for (int64_t k = first; k < first + count; k++) {
        int64_t i = g_bvh.idx[k];
        const int32_t *t = sc->tris + 3 * i;
        for (int c = 0; c < 3; c++)
            for (int a = 0; a < 3; a++) {
                double x = (double)sc->verts[3 * (int64_t)t[c] + a];
                if (x < nd->lo[a]) nd->lo[a] = x;
                if (x > nd->hi[a]) nd->hi[a] = x;
            }
        for (int a = 0; a < 3; a++) {
            double x = g_bvh.cent[3 * i + a];
            if (x < clo[a]) clo[a] = x;
            if (x > chi[a]) chi[a] = x;
        }
    }
    for (int a = 0; a < 3; a++) { nd->lo[a] -= 1e-6; nd->hi[a] += 1e-6; }
    if (count <= 4) {
        nd->left = nd->right = -1; nd->first = first; nd->count = count;
        return me;
    }
    int axis = 0;
    for (int a = 1; a < 3; a++)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    g_sort_axis = axis;
    qsort(g_bvh.idx + first, (size_t)count, sizeof(int64_t), cmp_cent);
    int64_t half = count / 2;
    nd->first = -1; nd->count = 0;
    int64_t l = bvh_build_rec(sc, first, half);
    int64_t r = bvh_build_rec(sc, first + half, count - half);
    g_bvh.nodes[me].left = l;
    g_bvh.nodes[me].right = r;
    return me;
}

static void bvh_free(void)
{
    free(g_bvh.nodes); free(g_bvh.idx); free(g_bvh.cent);
    memset(&g_bvh, 0, sizeof(g_bvh));
    g_bvh_scene = NULL;
}

static int bvh_build(const orc_scene *sc)
{
    bvh_free();
    int64_t nt = sc->nt;
    if (nt == 0) { g_bvh_scene = sc; return 0; }
    g_bvh.nodes = (onode *)calloc((size_t)(2 * nt), sizeof(onode));
    g_bvh.idx = (int64_t *)malloc((size_t)nt * sizeof(int64_t));
    g_bvh.cent = (double *)malloc((size_t)nt * 3 * sizeof(double));
    if (!g_bvh.nodes || !g_bvh.idx || !g_bvh.cent) { bvh_free(); return -1; }
    for (int64_t i = 0; i < nt; i++) {
        g_bvh.idx[i] = i;
        vec3 v0, v1, v2;
        tri_verts(sc, i, &v0, &v1, &v2);
        g_bvh.cent[3 * i + 0] = (v0.x + v1.x + v2.x) / 3.0;
        g_bvh.cent[3 * i + 1] = (v0.y + v1.y + v2.y) / 3.0;
        g_bvh.cent[3 * i + 2] = (v0.z + v1.z + v2.z) / 3.0;
    }
    bvh_build_rec(sc, 0, nt);
    g_bvh_scene = sc;
    return 0;
}

static int box_overlaps(const onode *nd, vec3 o, vec3 d, double tmax)
{
    double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    double t0 = 0.0, t1 = tmax * (1.0 + 1e-12) + 1e-9;
    for (int a = 0; a < 3; a++) {
        if (dd[a] == 0.0) {
            if (oo[a] < nd->lo[a] || oo[a] > nd->hi[a]) return 0;
            continue;
        }
        double ta = (nd->lo[a] - oo[a]) / dd[a];
        double tb = (nd->hi[a] - oo[a]) / dd[a];
        if (ta > tb) { double s = ta; ta = tb; tb = s; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

static int64_t closest_bvh(const orc_scene *sc, vec3 o, vec3 d, int64_t skip, double *t_best)
{
    int64_t best = -1;
    double tb = INFINITY;
    if (sc->nt == 0) { *t_best = tb; return -1; }
    int64_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const onode *nd = &g_bvh.nodes[stack[--sp]];
        if (!box_overlaps(nd, o, d, tb)) continue;
        if (nd->left < 0) {
            for (int64_t k = nd->first; k < nd->first + nd->count; k++) {
                int64_t i = g_bvh.idx[k];
                if (i == skip) continue;
                vec3 v0, v1, v2;
                double t;
                tri_verts(sc, i, &v0, &v1, &v2);
                if (mt_hit(o, d, v0, v1, v2, &t) && (t < tb || (t == tb && i < best))) {
                    tb = t; best = i;
                }
            }
        } else {
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
    *t_best = tb;
    return best;
}

static int g_use_bvh = 0;

static int64_t closest(const orc_scene *sc, vec3 o, vec3 d, int64_t skip, double *t_best)
{
    if (g_use_bvh) return closest_bvh(sc, o, d, skip, t_best);
    return closest_brute(sc, o, d, skip, t_best);
}

/* exposed for the tests: closest hit of a single ray */
int64_t orc_closest(const orc_scene *sc, const double o[3], const double d[3], int64_t skip,
                    int use_bvh, double *t_best)
{
    if (use_bvh && g_bvh_scene != sc && bvh_build(sc) != 0) return -2;
    g_use_bvh = use_bvh;
    return closest(sc, vload3d(o), vload3d(d), skip, t_best);
}

/* ------------------------------------------------------------------------ */
/* material: Eqs. (1)-(3)                                                    */
/* ------------------------------------------------------------------------ */

/* n: unit face normal flipped against the incident direction d.
 * u0,u1: two uniforms for the random point r on the unit sphere.
 * Returns the unit outgoing direction t_o,c. */
static vec3 bounce_dir(vec3 d, vec3 n, double alpha, double u0, double u1)
{
    /* Eq. 2, law of reflection */
    double dn = vdot(d, n);
    double s2 = 2.0 * dn;
    vec3 m = mk(d.x - s2 * n.x, d.y - s2 * n.y, d.z - s2 * n.z);
    /* Eq. 1: n + r with r uniform on the unit sphere (Archimedes' z, phi) */
    double z = 1.0 - 2.0 * u0;
    double rho = sqrt(fmax(0.0, 1.0 - z * z));
    double sp, cp;
    orc_sincos_turn(u1, &sp, &cp);
    vec3 td = mk(n.x + rho * cp, n.y + rho * sp, n.z + z);
    double tl = vlen(td);
    td = (tl < 1e-12) ? n : vdiv(td, tl);
    /* Eq. 3 blend, renormalised */
    double b = 1.0 - alpha;
    vec3 tc = mk(alpha * td.x + b * m.x, alpha * td.y + b * m.y, alpha * td.z + b * m.z);
    double cl = vlen(tc);
    return (cl < 1e-12) ? m : vdiv(tc, cl);
}

vec3 orc_face_normal(const orc_scene *sc, int64_t tri, vec3 d)
{
    vec3 v0, v1, v2;
    tri_verts(sc, tri, &v0, &v1, &v2);
    vec3 n = vcross(vsub(v1, v0), vsub(v2, v0));
    n = vdiv(n, vlen(n));
    if (vdot(n, d) > 0.0) n = mk(-n.x, -n.y, -n.z);
    return n;
}

/* exposed for the tests */
void orc_bounce(const double d[3], const double n[3], double alpha, double u0, double u1, double out[3])
{
    vec3 r = bounce_dir(vload3d(d), vload3d(n), alpha, u0, u1);
    out[0] = r.x; out[1] = r.y; out[2] = r.z;
}

/* ------------------------------------------------------------------------ */
/* tracing                                                                   */
/* ------------------------------------------------------------------------ */

#define INV_2PI 0.15915494309189535

/* pieces of the per-triangle launch (built by build_pieces below) */
typedef struct {
    vec3 v[3];
    int64_t parent;
} orc_piece;

static orc_piece *g_pieces;
static int64_t g_n_pieces, g_cap_pieces;

typedef struct {
    int64_t n_src, n_per_src;        /* rays per source */
    int64_t n_virt_per_src;          /* rays + points per source */
    vec3 oT, oR;
    double at, bt, slo, shi, omega;
    double c0, s0, c1, s1;           /* cos, sin of the azimuth bounds */
} trace_setup;

static vec3 centroid(const double *p, int32_t n)
{
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int32_t i = 0; i < n; i++) { sx += p[3 * i]; sy += p[3 * i + 1]; sz += p[3 * i + 2]; }
    return mk(sx / (double)n, sy / (double)n, sz / (double)n);
}

static void setup(const orc_scene *sc, const orc_array *ar, const orc_trace_params *tp, trace_setup *s)
{
    s->n_src = ar->shared ? 1 : ar->ntx;
    if (tp->tri_g > 0)
        s->n_per_src = g_n_pieces * (int64_t)tp->tri_g * tp->tri_g;
    else
        s->n_per_src = ar->shared ? tp->n_rays : tp->n_rays / ar->ntx;
    s->n_virt_per_src = s->n_per_src + sc->npts;
    s->oT = centroid(ar->tx, ar->ntx);
    s->oR = centroid(ar->rx, ar->nrx);
    s->at = tp->az_min * INV_2PI;
    s->bt = tp->az_max * INV_2PI;
    s->slo = sin(tp->el_min);
    s->shi = sin(tp->el_max);
    s->omega = (tp->az_max - tp->az_min) * (s->shi - s->slo);
    s->c0 = cos(tp->az_min);
    s->s0 = sin(tp->az_min);
    s->c1 = cos(tp->az_max);
    s->s1 = sin(tp->az_max);
}

/* Per-triangle casting (Sec. III: many rays are cast towards each mesh
 * triangle).  Ray i of a source aims at triangle f = i / g^2; its index
 * k = i mod g^2 picks cell (k mod g, k / g) of a g x g grid over the unit
 * square, (u1, u2) is uniform in that cell and the area-preserving map
 * x = (1 - sqrt u1) v0 + sqrt u1 (1 - u2) v1 + sqrt u1 u2 v2 puts it on the
 * triangle, so the rays are uniform over the triangle's area and stratified.
 * A point uniform over area A seen from src has the solid-angle density
 * d^2 / (A |cos theta|), so the weight p0 A |cos theta| / d^2 (p0 = 1 / solid
 * angle of the field of view; A |cos theta| = |n_area . dir| / 2) makes the
 * sum over triangles estimate the same mean as the uniform launch, provided
 * every direction is counted once: a ray counts only if its first hit is the
 * triangle it aims at, and rays outside the field of view are not traced
 * (reading: the field of view is the same azimuth / elevation box as the
 * uniform launch; the azimuth test below needs a span of at most pi).
 * Returns 0 for a ray that is not traced. */
/* Pieces of the per-triangle launch: every triangle (in upload order), cut
 * by midpoint subdivision into four while the piece subtends more than
 * omega_max steradians from the Tx phase centre o (and depth < depth_max);
 * children in the order (v0, m01, m20), (m01, v1, m12), (m20, m12, v2),
 * (m01, m12, m20), depth first; pieces no ray of which can enter the field
 * of view are dropped (below).  A piece keeps its parent triangle, the one
 * its rays must hit first.  With omega_max = 0 the pieces are the triangles
 * in view.
 * Any subdivision leaves the estimate unbiased (every ray is weighted by its
 * own piece's area); it only moves rays towards the triangles that fill the
 * most solid angle, where area-uniform points on a large triangle would be
 * sparse (the near-field ground). */
/* solid angle of triangle (a, b, c) seen from o (Van Oosterom and Strackee 1983) */
static double tri_solid_angle(vec3 a, vec3 b, vec3 c, vec3 o)
{
    vec3 x = vsub(a, o), y = vsub(b, o), z = vsub(c, o);
    double lx = vlen(x), ly = vlen(y), lz = vlen(z);
    double num = fabs(vdot(x, vcross(y, z)));
    double den = lx * ly * lz + vdot(x, y) * lz + vdot(x, z) * ly + vdot(y, z) * lx;
    return 2.0 * atan2(num, den);
}

static vec3 mid(vec3 a, vec3 b) { return mk((a.x + b.x) * 0.5, (a.y + b.y) * 0.5, (a.z + b.z) * 0.5); }

static int push_piece(vec3 a, vec3 b, vec3 c, int64_t parent)
{
    if (g_n_pieces == g_cap_pieces) {
        int64_t cap = g_cap_pieces ? 2 * g_cap_pieces : 1024;
        orc_piece *p = (orc_piece *)realloc(g_pieces, (size_t)cap * sizeof(orc_piece));
        if (!p) return -1;
        g_pieces = p;
        g_cap_pieces = cap;
    }
    orc_piece *q = &g_pieces[g_n_pieces++];
    q->v[0] = a; q->v[1] = b; q->v[2] = c;
    q->parent = parent;
    return 0;
}

/* The field of view as seen from the launch's sources (the Tx phase centre,
 * or every Tx element), to drop pieces none of whose rays can count: a ray
 * outside the field of view is not traced, so a piece whose every point lies
 * outside it, from every source, only takes up ray indices.  The test is
 * conservative: all three vertices beyond the same bounding plane of the
 * azimuth wedge, or inside the same excluded elevation cone where that cone
 * is convex (below el_min <= 0, above el_max >= 0), by a margin of 1e-9 of
 * their distance (far above the rounding of a ray's direction); the excluded
 * regions are convex, so then every point of the piece is outside. */
typedef struct {
    const double *src;
    int32_t n_src;
    double c0, s0, c1, s1;           /* cos, sin of the azimuth bounds */
    double slo, shi;                 /* sin of the elevation bounds */
} fov_cull;

#define CULL_EPS 1e-9

static int beyond_fov(vec3 a, vec3 b, vec3 c, vec3 src, const fov_cull *f)
{
    vec3 r[3] = {vsub(a, src), vsub(b, src), vsub(c, src)};
    int n0 = 0, n1 = 0, n2 = 0, n3 = 0;
    for (int k = 0; k < 3; k++) {
        double l = vlen(r[k]);
        if (f->c0 * r[k].y - f->s0 * r[k].x < -CULL_EPS * l) n0++;
        if (f->c1 * r[k].y - f->s1 * r[k].x > CULL_EPS * l) n1++;
        if (r[k].z < f->slo * l - CULL_EPS * l) n2++;
        if (r[k].z > f->shi * l + CULL_EPS * l) n3++;
    }
    return n0 == 3 || n1 == 3 || (f->slo <= 0.0 && n2 == 3) || (f->shi >= 0.0 && n3 == 3);
}

static int outside_fov(vec3 a, vec3 b, vec3 c, const fov_cull *f)
{
    for (int32_t t = 0; t < f->n_src; t++)
        if (!beyond_fov(a, b, c, mk(f->src[3 * t], f->src[3 * t + 1], f->src[3 * t + 2]), f))
            return 0;
    return 1;
}

static int cut(vec3 a, vec3 b, vec3 c, int64_t parent, vec3 o, double omega_max, int depth,
               int depth_max, const fov_cull *fov)
{
    if (omega_max > 0.0 && depth < depth_max && tri_solid_angle(a, b, c, o) > omega_max) {
        vec3 ab = mid(a, b), bc = mid(b, c), ca = mid(c, a);
        if (cut(a, ab, ca, parent, o, omega_max, depth + 1, depth_max, fov)) return -1;
        if (cut(ab, b, bc, parent, o, omega_max, depth + 1, depth_max, fov)) return -1;
        if (cut(ca, bc, c, parent, o, omega_max, depth + 1, depth_max, fov)) return -1;
        return cut(ab, bc, ca, parent, o, omega_max, depth + 1, depth_max, fov);
    }
    if (fov && outside_fov(a, b, c, fov)) return 0;
    return push_piece(a, b, c, parent);
}

/* fov: NULL keeps every piece */
static int build_pieces(const orc_scene *sc, vec3 o, double omega_max, int depth_max,
                        const fov_cull *fov)
{
    g_n_pieces = 0;
    for (int64_t f = 0; f < sc->nt; f++) {
        vec3 v0, v1, v2;
        tri_verts(sc, f, &v0, &v1, &v2);
        if (cut(v0, v1, v2, f, o, omega_max, 0, depth_max, fov)) return -1;
    }
    return 0;
}

/* the culling of a launch with field of view (az_min, az_max, el_min, el_max)
 * from the array's sources; o: the Tx phase centre (the shared source) */
static void make_cull(const orc_array *ar, const double *o, double az_min, double az_max,
                      double el_min, double el_max, fov_cull *f)
{
    f->src = ar->shared ? o : ar->tx;
    f->n_src = ar->shared ? 1 : ar->ntx;
    f->c0 = cos(az_min);
    f->s0 = sin(az_min);
    f->c1 = cos(az_max);
    f->s1 = sin(az_max);
    f->slo = sin(el_min);
    f->shi = sin(el_max);
}

/* exposed for the tests: number of pieces and the vertices / parent of each;
 * fov = (az_min, az_max, el_min, el_max) of the launch, or NULL for no
 * culling */
int64_t orc_pieces(const orc_scene *sc, const orc_array *ar, double omega_max, int32_t depth_max,
                   const double *fov, double *verts, int64_t *parent, int64_t cap)
{
    vec3 o = centroid(ar->tx, ar->ntx);
    double oc[3] = {o.x, o.y, o.z};
    fov_cull f;
    if (fov) make_cull(ar, oc, fov[0], fov[1], fov[2], fov[3], &f);
    if (build_pieces(sc, o, omega_max, depth_max, fov ? &f : NULL)) return -1;
    for (int64_t i = 0; i < g_n_pieces && i < cap; i++) {
        for (int k = 0; k < 3; k++) {
            verts[9 * i + 3 * k] = g_pieces[i].v[k].x;
            verts[9 * i + 3 * k + 1] = g_pieces[i].v[k].y;
            verts[9 * i + 3 * k + 2] = g_pieces[i].v[k].z;
        }
        parent[i] = g_pieces[i].parent;
    }
    return g_n_pieces;
}

static int launch_tri(const orc_scene *sc, const orc_trace_params *tp, const trace_setup *s,
                      vec3 src, int64_t i, int64_t t, vec3 *dir, double *w)
{
    (void)sc;
    int64_t g = tp->tri_g, gg = g * g;
    int64_t f = i / gg, k = i % gg;
    double u[4];
    draw(tp->seed, (uint64_t)i, (uint64_t)t, 0, u);
    double u1 = ((double)(k % g) + u[0]) / (double)g;
    double u2 = ((double)(k / g) + u[1]) / (double)g;
    vec3 v0 = g_pieces[f].v[0], v1 = g_pieces[f].v[1], v2 = g_pieces[f].v[2];
    double su = sqrt(u1);
    double b0 = 1.0 - su, b1 = su * (1.0 - u2), b2 = su * u2;
    vec3 x = mk(b0 * v0.x + b1 * v1.x + b2 * v2.x, b0 * v0.y + b1 * v1.y + b2 * v2.y,
                b0 * v0.z + b1 * v1.z + b2 * v2.z);
    vec3 a = vsub(x, src);
    double d2 = vdot(a, a);
    if (!(d2 > 0.0)) return 0;
    vec3 d = vdiv(a, sqrt(d2));
    if (!(d.z >= s->slo && d.z <= s->shi)) return 0;
    if (!(s->c0 * d.y - s->s0 * d.x >= 0.0 && s->c1 * d.y - s->s1 * d.x <= 0.0)) return 0;
    vec3 na = vcross(vsub(v1, v0), vsub(v2, v0));
    *w = (0.5 * fabs(vdot(na, d))) / (d2 * s->omega);
    if (!(*w > 0.0)) return 0;
    *dir = d;
    return 1;
}

/* first bin b with u < cdf[b+1] */
static int32_t cdf_bin(const double *cdf, int32_t nb, double u)
{
    int32_t lo = 0, hi = nb - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi) / 2;
        if (u < cdf[mid + 1]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* launch direction and weight of ray i of source t (Sec. III-A: each
 * transmitter sends out many rays; uniform in solid angle over the field of
 * view, or drawn from a binned proposal with weight p0/q). */
static vec3 launch(const orc_trace_params *tp, const trace_setup *s, int64_t i, int64_t t, double *w)
{
    double u[4];
    draw(tp->seed, (uint64_t)i, (uint64_t)t, 0, u);
    double fa, fs;
    if (tp->cdf == NULL) {
        fa = u[0]; fs = u[1]; *w = 1.0;
    } else {
        int32_t nb = tp->n_az * tp->n_el;
        int32_t b = cdf_bin(tp->cdf, nb, u[0]);
        int32_t ia = b % tp->n_az, ie = b / tp->n_az;
        fa = ((double)ia + u[1]) / (double)tp->n_az;
        fs = ((double)ie + u[2]) / (double)tp->n_el;
        double q = tp->cdf[b + 1] - tp->cdf[b];
        *w = 1.0 / ((double)nb * q);
    }
    double turn = s->at + fa * (s->bt - s->at);
    double sz = s->slo + fs * (s->shi - s->slo);
    double ce = sqrt(1.0 - sz * sz);
    double sa, ca;
    orc_sincos_turn(turn, &sa, &ca);
    return mk(ce * ca, ce * sa, sz);
}

/* exposed for the tests: launch direction of a ray */
void orc_launch_dir(const orc_scene *sc, const orc_array *ar, const orc_trace_params *tp,
                    int64_t i, int64_t t, double out[4])
{
    trace_setup s;
    setup(sc, ar, tp, &s);
    double w;
    vec3 d = launch(tp, &s, i, t, &w);
    out[0] = d.x; out[1] = d.y; out[2] = d.z; out[3] = w;
}

static int emit(orc_path *paths, int64_t cap, int64_t *np, const orc_path *p)
{
    if (*np < cap && paths) paths[*np] = *p;
    (*np)++;
    return 0;
}

/* The bounces of one ray leaving o along the unit vector dir (Sec. III-A):
 * closest hit, reception of every segment that follows a hit (reading R15:
 * its closest approach to the Rx phase centre oR lies ahead, before the next
 * hit, inside the sphere of radius sqrt(r2)), and at each hit the new
 * direction of Eqs. 1-3 with the random numbers of counter (i, t, j + 1).
 * pa carries src, ray and amp; its hit points are filled in here.  target >= 0:
 * the ray is dropped (no hits recorded, no paths) unless its first hit is that
 * triangle. */
static void trace_from(const orc_scene *sc, vec3 oR, uint64_t seed, int32_t B, double r2, vec3 o,
                       vec3 dir, int64_t i, int64_t t, int64_t target, orc_path *pa, int32_t *hrow,
                       orc_path *paths, int64_t cap, int64_t *np)
{
    double L = 0.0;
    int64_t prev = -1;
    for (int32_t j = 0; j <= B; j++) {
        double th;
        int64_t h = closest(sc, o, dir, prev, &th);
        /* a ray cast towards a triangle counts only if that triangle is its first hit */
        if (j == 0 && target >= 0 && h != target) return;
        if (hrow) hrow[j] = (int32_t)h;
        if (j >= 1) {
            vec3 w2 = vsub(oR, o);
            double ts = vdot(w2, dir);
            if (ts > 0.0 && ts < th) {
                double cx = (o.x + ts * dir.x) - oR.x;
                double cy = (o.y + ts * dir.y) - oR.y;
                double cz = (o.z + ts * dir.z) - oR.z;
                if (cx * cx + cy * cy + cz * cz <= r2) {
                    pa->K = j;
                    pa->L = L;
                    emit(paths, cap, np, pa);
                }
            }
        }
        if (h < 0 || j == B) break;
        vec3 p = mk(o.x + th * dir.x, o.y + th * dir.y, o.z + th * dir.z);
        L += th;
        pa->tri[j] = (int32_t)h;
        pa->vid[j] = sc->tri_obj[h];
        pa->p[j][0] = p.x; pa->p[j][1] = p.y; pa->p[j][2] = p.z;
        vec3 n = orc_face_normal(sc, h, dir);
        double u[4];
        draw(seed, (uint64_t)i, (uint64_t)t, (uint64_t)(j + 1), u);
        /* material mix of Eq. 3: the face's own value when faces carry one */
        double alpha = sc->tri_alpha ? (double)sc->tri_alpha[h] : (double)sc->obj_alpha[sc->tri_obj[h]];
        dir = bounce_dir(dir, n, alpha, u[0], u[1]);
        o = p;
        prev = h;
    }
}

/* Trace the listed virtual rays (all of them when vids == NULL).
 * Virtual ray v of source t = v / (n_per_src + npts): index i = v mod that;
 * i < n_per_src is a launched ray, otherwise point reflector i - n_per_src.
 * hits (optional): [n][max_bounces+1] closest-hit triangle of each traced
 * segment, -1 for a miss or a segment not traced.
 * Paths are emitted in (virtual ray, bounce) order; the count is returned in
 * *n_paths even when it exceeds cap. */
int orc_trace(const orc_scene *sc, const orc_array *ar, const orc_trace_params *tp, int use_bvh,
              const int64_t *vids, int64_t n_vids, int32_t *hits, orc_path *paths, int64_t cap,
              int64_t *n_paths)
{
    if (tp->max_bounces < 1 || tp->max_bounces > ORC_KMAX) return -1;
    if (ar->ntx < 1 || ar->nrx < 1) return -1;
    if (tp->tri_g < 0 || (tp->tri_g > 0 && !(tp->az_max - tp->az_min <= ORC_PI))) return -1;
    if (tp->tri_g > 0 && (tp->tri_omega_max < 0.0 || tp->tri_depth_max < 0 || tp->tri_depth_max > 20))
        return -1;
    if (tp->tri_g > 0) {
        vec3 o = centroid(ar->tx, ar->ntx);
        double oc[3] = {o.x, o.y, o.z};
        fov_cull f;
        make_cull(ar, oc, tp->az_min, tp->az_max, tp->el_min, tp->el_max, &f);
        if (build_pieces(sc, o, tp->tri_omega_max, tp->tri_depth_max, &f)) return -2;
    }
    trace_setup s;
    setup(sc, ar, tp, &s);
    if (use_bvh && g_bvh_scene != sc && bvh_build(sc) != 0) return -2;
    g_use_bvh = use_bvh;
    int64_t total = s.n_src * s.n_virt_per_src;
    int64_t n = vids ? n_vids : total;
    int32_t B = tp->max_bounces;
    double r2 = ar->rx_radius * ar->rx_radius;
    int64_t np = 0;
    for (int64_t k = 0; k < n; k++) {
        int64_t v = vids ? vids[k] : k;
        if (v < 0 || v >= total) return -1;
        int64_t t = v / s.n_virt_per_src, i = v % s.n_virt_per_src;
        vec3 src = ar->shared ? s.oT : vload3d(ar->tx + 3 * t);
        int32_t *hrow = hits ? hits + k * (B + 1) : NULL;
        if (hrow) for (int j = 0; j <= B; j++) hrow[j] = -1;
        orc_path pa;
        memset(&pa, 0, sizeof(pa));
        pa.src = ar->shared ? -1 : (int32_t)t;
        pa.ray = v;
        for (int j = 0; j < ORC_KMAX; j++) { pa.tri[j] = -1; pa.vid[j] = -1; }
        if (i >= s.n_per_src) {
            /* point reflector: one single-bounce path if both legs are clear */
            int64_t q = i - s.n_per_src;
            vec3 Q = vload3d(sc->pt_pos + 3 * q);
            vec3 a = vsub(Q, src);
            double la = vlen(a);
            vec3 b = vsub(s.oR, Q);
            double lb = vlen(b);
            double th;
            closest(sc, src, vdiv(a, la), -1, &th);
            if (th < la) continue;
            closest(sc, Q, vdiv(b, lb), -1, &th);
            if (th < lb) continue;
            pa.K = 1;
            pa.vid[0] = sc->nobj + (int32_t)q;
            pa.p[0][0] = Q.x; pa.p[0][1] = Q.y; pa.p[0][2] = Q.z;
            pa.L = la;
            pa.amp = sc->pt_ap[q] / (la * la * s.omega);
            emit(paths, cap, &np, &pa);
            continue;
        }
        double w;
        vec3 dir;
        int64_t target = -1;
        if (tp->tri_g > 0) {
            if (!launch_tri(sc, tp, &s, src, i, t, &dir, &w)) continue;
            pa.amp = w / (double)((int64_t)tp->tri_g * tp->tri_g);
            target = g_pieces[i / ((int64_t)tp->tri_g * tp->tri_g)].parent;
        } else {
            dir = launch(tp, &s, i, t, &w);
            pa.amp = w / (double)s.n_per_src;
        }
        trace_from(sc, s.oR, tp->seed, B, r2, src, dir, i, t, target, &pa, hrow, paths, cap, &np);
    }
    *n_paths = np;
    return 0;
}

/* Trace n caller-supplied rays (Sec. III-A launches rays from each
 * transmitter; here the caller picks them): ray i starts at orig[i] along
 * dir[i] (normalised here), every path it produces has amplitude amp[i] and
 * source src[i] (-1 for a shared launch, else a Tx index in [0, ntx),
 * ascending over i).  The bounce at hit j uses the random numbers of counter
 * (i - i0, max(src[i], 0), j + 1), i0 the first ray of the same source: so
 * the launch's own rays reproduce orc_trace exactly.  No point reflectors.  Paths are emitted in
 * (ray, bounce) order with ray = i; hits as in orc_trace.  Returns -1 for an
 * invalid source list or a non-finite or zero vector. */
int orc_trace_rays(const orc_scene *sc, const orc_array *ar, int use_bvh, int64_t n,
                   const double *orig, const double *dir, const double *amp, const int32_t *src,
                   int32_t max_bounces, uint64_t seed, int32_t *hits, orc_path *paths, int64_t cap,
                   int64_t *n_paths)
{
    if (max_bounces < 1 || max_bounces > ORC_KMAX || n < 0) return -1;
    if (ar->ntx < 1 || ar->nrx < 1) return -1;
    for (int64_t i = 0; i < n; i++) {
        int32_t t = src[i];
        if (ar->shared ? t != -1 : (t < 0 || t >= ar->ntx || (i > 0 && t < src[i - 1]))) return -1;
        for (int a = 0; a < 3; a++)
            if (!isfinite(orig[3 * i + a]) || !isfinite(dir[3 * i + a])) return -1;
        if (!isfinite(amp[i])) return -1;
        if (dir[3 * i] == 0.0 && dir[3 * i + 1] == 0.0 && dir[3 * i + 2] == 0.0) return -1;
    }
    if (use_bvh && g_bvh_scene != sc && bvh_build(sc) != 0) return -2;
    g_use_bvh = use_bvh;
    vec3 oR = centroid(ar->rx, ar->nrx);
    double r2 = ar->rx_radius * ar->rx_radius;
    int32_t B = max_bounces;
    int64_t np = 0;
    int64_t i0 = 0;
    for (int64_t i = 0; i < n; i++) {
        if (i > 0 && src[i] != src[i - 1]) i0 = i;
        int32_t *hrow = hits ? hits + i * (B + 1) : NULL;
        if (hrow) for (int j = 0; j <= B; j++) hrow[j] = -1;
        orc_path pa;
        memset(&pa, 0, sizeof(pa));
        pa.src = src[i];
        pa.ray = i;
        pa.amp = amp[i];
        for (int j = 0; j < ORC_KMAX; j++) { pa.tri[j] = -1; pa.vid[j] = -1; }
        vec3 d = vload3d(dir + 3 * i);
        d = vdiv(d, vlen(d));
        trace_from(sc, oR, seed, B, r2, vload3d(orig + 3 * i), d, i - i0, src[i] > 0 ? src[i] : 0,
                   -1, &pa, hrow, paths, cap, &np);
    }
    *n_paths = np;
    return 0;
}

void orc_release(void) { bvh_free(); }

/* ------------------------------------------------------------------------ */
/* synthesis: Eq. (4) with the FMCW instantaneous frequency                  */
/* ------------------------------------------------------------------------ */

#define C0 299792458.0

static vec3 moved(const orc_scene *sc, const orc_path *p, int j, double tau)
{
    const double *v = (p->vid[j] < sc->nobj) ? sc->obj_vel + 3 * p->vid[j]
                                             : sc->pt_vel + 3 * (p->vid[j] - sc->nobj);
    return mk(p->p[j][0] + v[0] * tau, p->p[j][1] + v[1] * tau, p->p[j][2] + v[2] * tau);
}

/* internal length p_1 -> ... -> p_K at time tau */
static double inner_len(const orc_scene *sc, const orc_path *p, double tau)
{
    double L = 0.0;
    for (int j = 0; j + 1 < p->K; j++) L += vlen(vsub(moved(sc, p, j + 1, tau), moved(sc, p, j, tau)));
    return L;
}

/* model 0 (exact): d = |p_1(m) - tx_t| + inner(m) + |rx_r - p_K(m)|,
 *                  term = amp exp(-j 2 pi f_k d / c)
 * model 1 (separable): term = amp exp(-j 2 pi [f0 (dT + dR) + f_k D(m)] / c)
 *   with D(m) = |p_1(m) - o_s| + inner(m) + |o_R - p_K(m)| (o_s = Tx of the
 *   path, or the Tx phase centre for a shared launch), dT = |p_1 - tx_t| -
 *   |p_1 - o_s| and dR = |rx_r - p_K| - |o_R - p_K| at chirp 0.
 * Entries are flat indices c*M*K + m*K + k; idx == NULL means the full cube.
 * out: [n][2] (re, im). */
int orc_synth(const orc_path *paths, int64_t np, const orc_scene *sc, const orc_array *ar,
              const orc_chirp *ch, int model, const int64_t *idx, int64_t n_idx, double *out)
{
    int64_t M = ch->n_chirps, K = ch->n_samples;
    int64_t C = (int64_t)ar->ntx * ar->nrx;
    int64_t n = idx ? n_idx : C * M * K;
    vec3 oT = centroid(ar->tx, ar->ntx), oR = centroid(ar->rx, ar->nrx);
    for (int64_t e = 0; e < n; e++) {
        int64_t f = idx ? idx[e] : e;
        if (f < 0 || f >= C * M * K) return -1;
        int64_t c = f / (M * K), m = (f / K) % M, k = f % K;
        int64_t t = c / ar->nrx, r = c % ar->nrx;
        vec3 tx = vload3d(ar->tx + 3 * t), rx = vload3d(ar->rx + 3 * r);
        double fk = ch->f0 + ch->bandwidth * (double)k / (double)K;
        double tau = (double)m * ch->t_rep;
        double re = 0.0, im = 0.0;
        for (int64_t pi = 0; pi < np; pi++) {
            const orc_path *p = &paths[pi];
            if (p->src >= 0 && p->src != t) continue;
            vec3 P1 = moved(sc, p, 0, tau), PK = moved(sc, p, p->K - 1, tau);
            double inner = inner_len(sc, p, tau);
            double phase;
            if (model == 0) {
                double d = vlen(vsub(P1, tx)) + inner + vlen(vsub(rx, PK));
                phase = fk * d / C0;
            } else {
                vec3 os = p->src >= 0 ? vload3d(ar->tx + 3 * p->src) : oT;
                vec3 p1 = moved(sc, p, 0, 0.0), pk = moved(sc, p, p->K - 1, 0.0);
                double dT = vlen(vsub(p1, tx)) - vlen(vsub(p1, os));
                double dR = vlen(vsub(rx, pk)) - vlen(vsub(oR, pk));
                double D = vlen(vsub(P1, os)) + inner + vlen(vsub(oR, PK));
                phase = (ch->f0 * (dT + dR) + fk * D) / C0;
            }
            double fr = phase - floor(phase);          /* exact */
            double ang = 6.283185307179586 * fr;
            re += p->amp * cos(ang);
            im -= p->amp * sin(ang);
        }
        out[2 * e] = re;
        out[2 * e + 1] = im;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* learned-proposal inputs                                                   */
/* ------------------------------------------------------------------------ */

/* Scene code: 16 azimuth sectors x 8 probe rays at elevation 0 from the Tx
 * phase centre, sector s ray i at azimuth fraction (8 s + i + 1/2) / 128 of
 * the field of view.  code[s] = mean over its rays of exp(-t / 10 m) when the
 * closest hit belongs to an object other than object 0 (the ground), else 0. */
int orc_probe(const orc_scene *sc, const orc_array *ar, const orc_trace_params *tp, int use_bvh,
              double code[16])
{
    trace_setup s;
    setup(sc, ar, tp, &s);
    if (use_bvh && g_bvh_scene != sc && bvh_build(sc) != 0) return -2;
    g_use_bvh = use_bvh;
    for (int k = 0; k < 16; k++) {
        double acc = 0.0;
        for (int i = 0; i < 8; i++) {
            double fa = ((double)(8 * k + i) + 0.5) / 128.0;
            double turn = s.at + fa * (s.bt - s.at);
            double sa, ca;
            orc_sincos_turn(turn, &sa, &ca);
            double th;
            int64_t h = closest(sc, s.oT, mk(ca, sa, 0.0), -1, &th);
            if (h >= 0 && sc->tri_obj[h] != 0) acc += exp(-th / 10.0);
        }
        code[k] = acc / 8.0;
    }
    return 0;
}

/* Bin (ie * n_az + ia) of the uniform launch of every traced ray, in hit-list
 * order (source-major): ia = floor(u0 n_az), ie = floor(u1 n_el). */
void orc_uniform_bins(uint64_t seed, int64_t n_per_src, int64_t n_src, int32_t n_az, int32_t n_el,
                      int32_t *bins)
{
    for (int64_t t = 0; t < n_src; t++)
        for (int64_t i = 0; i < n_per_src; i++) {
            double u[4];
            draw(seed, (uint64_t)i, (uint64_t)t, 0, u);
            int32_t ia = (int32_t)(u[0] * n_az), ie = (int32_t)(u[1] * n_el);
            if (ia >= n_az) ia = n_az - 1;
            if (ie >= n_el) ie = n_el - 1;
            bins[t * n_per_src + i] = ie * n_az + ia;
        }
}

/* ------------------------------------------------------------------------ */
/* imaging: delay-and-sum back-projection of a stepped-frequency cube        */
/* ------------------------------------------------------------------------ */

/* The textbook delay-and-sum image of a single-sweep cube (the paper forms
 * its hand images by brute-force back-projection; here written from the
 * definition): for voxel x,
 *   image(x) = sum_{t, r} sum_n s[t n_rx + r][n] exp(+j 2 pi f_n d / c),
 *   d = |x - tx_t| + |x - rx_r|,  f_n = f0 + n df,
 * the matched filter of the synthesis phase exp(-j 2 pi f_n d / c).
 * cube: [n_tx n_rx][nf][2] (re, im); vox: [nv][3]; out: [nv][2].  FP64,
 * one sin / cos per term. */

int orc_backproject(const orc_array *ar, double f0, double df, int32_t nf, const double *cube,
                    const double *vox, int64_t nv, double *out)
{
    if (ar->ntx < 1 || ar->nrx < 1 || nf < 1 || nv < 0) return -1;
    for (int64_t v = 0; v < nv; v++) {
        vec3 x = vload3d(vox + 3 * v);
        double re = 0.0, im = 0.0;
        for (int32_t t = 0; t < ar->ntx; t++) {
            double dt = vlen(vsub(x, vload3d(ar->tx + 3 * t)));
            for (int32_t r = 0; r < ar->nrx; r++) {
                double d = dt + vlen(vsub(x, vload3d(ar->rx + 3 * r)));
                const double *s = cube + 2 * ((int64_t)(t * ar->nrx + r) * nf);
                for (int32_t n = 0; n < nf; n++) {
                    double ph = 2.0 * ORC_PI * (f0 + (double)n * df) * d / C0;
                    double c = cos(ph), sn = sin(ph);
                    re += s[2 * n] * c - s[2 * n + 1] * sn;
                    im += s[2 * n] * sn + s[2 * n + 1] * c;
                }
            }
        }
        out[2 * v] = re;
        out[2 * v + 1] = im;
    }
    return 0;
}
