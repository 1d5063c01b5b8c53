// rr_host.cpp -- the C ABI of libradray: context, validation, device buffers
// and the launch sequence of the trace and synthesis kernels.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include "rr_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(RR_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grow to at least n bytes (contents are not preserved)
    int ensure(size_t n)
    {
        if (n <= bytes && p) return RR_OK;
        release();
        if (n == 0) n = 256;
        if (hipMalloc(&p, n) != hipSuccess) {
            p = nullptr;
            return fail(RR_ENOMEM, "hipMalloc(%zu) failed", n);
        }
        bytes = n;
        return RR_OK;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Device path list: one allocation, planes carved out of it.
struct PathStore {
    DevBuf buf;
    PathSoA soa;
    int alloc(int64_t cap)
    {
        if (cap < 1) cap = 1;
        if (soa.cap >= cap && buf.p) return RR_OK;
        size_t per = 4 + 4 + 8 + 4 + 4 * RR_KMAX + 4 * RR_KMAX + 8 * 3 * RR_KMAX + 8 + 8;
        int rc = buf.ensure((size_t)cap * per + 1024);
        if (rc) return rc;
        char *b = buf.as<char>();
        size_t off = 0;
        auto take = [&](size_t bytes) {
            char *r = b + off;
            off += (bytes + 255) & ~size_t(255);
            return r;
        };
        soa.cap = cap;
        soa.ray = (int64_t *)take(8 * cap);
        soa.p = (double *)take(8 * 3 * RR_KMAX * cap);
        soa.L = (double *)take(8 * cap);
        soa.amp = (double *)take(8 * cap);
        soa.src = (int32_t *)take(4 * cap);
        soa.K = (int32_t *)take(4 * cap);
        soa.loc = (int32_t *)take(4 * cap);
        soa.tri = (int32_t *)take(4 * RR_KMAX * cap);
        soa.vid = (int32_t *)take(4 * RR_KMAX * cap);
        if (off > buf.bytes) {
            // plane rounding exceeded the estimate: allocate exactly
            buf.release();
            int rc2 = buf.ensure(off);
            if (rc2) return rc2;
            soa.cap = 0;
            return alloc(cap);
        }
        return RR_OK;
    }
};

bool finite3(const double *p, int64_t n)
{
    for (int64_t i = 0; i < 3 * n; i++)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

// Scratch of rr_synthesize_noalloc: synthesis records of up to
// RR_NOALLOC_MAX_PATHS paths, then the path ranges of up to RR_NOALLOC_MAX_TX
// transmitter groups.  Each GPU holds its own copy from module load until the
// process ends.  Host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device (g_scratch_dev), never
// through the array's name.
#define NOALLOC_RANGES_OFF (((size_t)RR_NOALLOC_MAX_PATHS * sizeof(SynPath) + 255) / 256 * 256)
#define NOALLOC_BYTES (NOALLOC_RANGES_OFF + (size_t)(RR_NOALLOC_MAX_TX + 2) * 8)
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};

// once per device, with that device current
int scratch_init(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(RR_EUNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[dev]) return RR_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(RR_EHIP, "scratch symbol address: %s", hipGetErrorString(e));
    g_scratch_dev[dev] = p;
    return RR_OK;
}
}  // namespace

struct rr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // [0, 1] trace stage, [2, 3] synthesis, [4, 5] imaging, [6] end of the
    // tracing kernels within the trace stage
    hipEvent_t ev[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool trace_timed = false, synth_timed = false, image_timed = false;

    // scene
    bool has_scene = false;
    int64_t n_tris = 0;
    int nobj = 0, npts = 0;
    DevBuf nodes, ltris, obj_alpha, obj_vel, pt_pos, pt_vel, pt_ap;
    int bvh_depth = 0;

    // array
    bool has_array = false;
    int ntx = 0, nrx = 0, mode = RR_TX_PER_ELEMENT;
    double rx_radius = 0.25;
    std::vector<double> tx_h, rx_h;
    double oT[3] = {0, 0, 0}, oR[3] = {0, 0, 0};
    DevBuf tx, rx;

    // chirp
    bool has_chirp = false;
    rr_chirp chirp{};

    // trace state
    DevBuf counts, offsets, bsums, counter, total, err_flag, hits, cdf;
    PathStore tmp;
    int64_t tmp_cap = 0;
    PathStore paths;
    int64_t n_paths = -1;          // -1: none
    bool paths_pending = false;    // a trace without a host count: n_paths not read back yet
    int64_t pending_keep = 0;      // at most this many paths kept by that trace
    int64_t hits_elems = 0;
    bool hits_recorded = false;
    int n_az = 0, n_el = 0;        // proposal grid (cdf set)

    // synthesis scratch
    DevBuf syn, ranges;
    DevBuf gT, gR, gA, gB;     // GEMM operands

    // learned proposal
    DevBuf tri_obj;            // object of each triangle, by original id
    DevBuf tri_alpha;          // staging of per-face alpha for rr_scene_set_alpha
    // per-triangle launch: pieces (triangles cut by solid angle) and their parents
    DevBuf pieces_v, pieces_p;
    double cast_omega = 0.0;
    int cast_depth = 8;
    double cast_fov[4] = {0, 0, 0, 0};   // field of view the pieces were built for
    bool pieces_valid = false;
    int64_t n_pieces = 0;
    std::vector<float> h_verts;
    // refit of the BVH to moved vertices (rr_scene_update_vertices)
    DevBuf tris_dev, verts_dev, refit_order, ubox;
    DevBuf fq_xt, fq_yt, fq_amp, fq_src, fq_part;   // exact-model GEMM engine
    DevBuf order_cells, order_rc, order_idx;   // coherent ray order of a trace
    DevBuf bp_sf;              // cube slices in fragment layout (MFMA back-projection)
    std::vector<double> h_tx, h_rx;
    std::vector<int64_t> refit_levels;   // starts of the levels in refit_order, deepest first
    std::vector<int32_t> h_tris;
    int64_t n_verts = 0, n_nodes = 0;
    TraceArgs last{};          // arguments of the last trace (histogram)
    int64_t last_traced = 0;
    int last_sampler = -1;
    DevBuf mlp_p, mlp_m, mlp_v, mlp_g, mlp_acts, mlp_z, mlp_dz, mlp_d, mlp_loss, mlp_part;
    DevBuf tr_codes, tr_hist, tr_loss;   // minibatch staging of rr_proposal_train
    DevBuf bp_peak;                      // peak of the last maximum projection
    DevBuf trace_stats;                  // work counters of rr_trace_work
    bool mlp_ready = false;
    int mlp_step = 0;
};

namespace {

// The trace stage of rr_trace / rr_trace_rays: tracing kernels, scan of the
// per-ray counts, scatter into (ray, bounce) order; grows the temporary
// buffer and re-runs once if it overflowed.
// With n_paths_out == NULL nothing waits for the GPU: the scatter reads the
// path count on the device and keeps at most min(path_cap, buffer) paths;
// resolve_paths reads the count back when the host first needs it.
template <class Kernels>
int run_trace(rr_ctx *c, TraceArgs &A, int64_t V, int64_t nb, int64_t path_cap, Kernels kernels,
              int64_t *n_paths_out)
{
    int rc;
    c->paths_pending = false;
    if (!n_paths_out) {
        A.tmp = c->tmp.soa;
        HIPCHK(hipMemsetAsync(c->counter.p, 0, 8, c->stream));
        HIPCHK(hipMemsetAsync(c->err_flag.p, 0, 4, c->stream));
        HIPCHK(hipEventRecord(c->ev[0], c->stream));
        HIPCHK(kernels(A));
        HIPCHK(hipEventRecord(c->ev[6], c->stream));
        HIPCHK(launch_scan_u8(A.counts, V, c->offsets.as<uint32_t>(), c->bsums.as<uint32_t>(),
                              nb + 1, c->total.as<unsigned long long>(), c->stream));
        const int64_t keep = path_cap > 0 ? std::min(path_cap, c->tmp_cap) : c->tmp_cap;
        if ((rc = c->paths.alloc(std::max<int64_t>(keep, 1)))) return rc;
        HIPCHK(launch_scatter(c->tmp.soa, A.counter, c->tmp_cap, c->offsets.as<uint32_t>(),
                              c->paths.soa, keep, c->stream));
        HIPCHK(hipEventRecord(c->ev[1], c->stream));
        c->n_paths = -1;
        c->paths_pending = true;
        c->pending_keep = keep;
        c->trace_timed = true;
        c->last = A;
        g_err.clear();
        return RR_OK;
    }
    for (int attempt = 0; attempt < 2; attempt++) {
        A.tmp = c->tmp.soa;
        HIPCHK(hipMemsetAsync(c->counter.p, 0, 8, c->stream));
        HIPCHK(hipMemsetAsync(c->err_flag.p, 0, 4, c->stream));
        HIPCHK(hipEventRecord(c->ev[0], c->stream));
        HIPCHK(kernels(A));
        HIPCHK(hipEventRecord(c->ev[6], c->stream));
        HIPCHK(launch_scan_u8(A.counts, V, c->offsets.as<uint32_t>(), c->bsums.as<uint32_t>(),
                              nb + 1, c->total.as<unsigned long long>(), c->stream));
        unsigned long long cnt = 0;
        int errf = 0;
        HIPCHK(hipMemcpyAsync(&cnt, c->counter.p, 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(&errf, c->err_flag.p, 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (errf)
            return fail(RR_EUNSUPPORTED, "traversal stack overflow (BVH depth %d)", c->bvh_depth);
        if ((int64_t)cnt > c->tmp_cap) {
            c->tmp_cap = (int64_t)cnt + cnt / 4 + 1024;
            if ((rc = c->tmp.alloc(c->tmp_cap))) return rc;
            continue;
        }
        int64_t keep = (int64_t)cnt;
        if (path_cap > 0 && keep > path_cap) keep = path_cap;
        if ((rc = c->paths.alloc(std::max<int64_t>(keep, 1)))) return rc;
        HIPCHK(launch_scatter(c->tmp.soa, A.counter, c->tmp_cap, c->offsets.as<uint32_t>(),
                              c->paths.soa, keep, c->stream));
        HIPCHK(hipEventRecord(c->ev[1], c->stream));
        c->n_paths = keep;
        c->trace_timed = true;
        c->last = A;
        if (n_paths_out) *n_paths_out = keep;
        g_err.clear();
        return RR_OK;
    }
    return fail(RR_EOVERFLOW, "temporary path buffer overflow persisted");
}

// The path count of a trace that did not read it back: one synchronisation.
// A count beyond the temporary buffer means records were dropped: the buffer
// grows for the next trace and RR_EOVERFLOW is returned.
int resolve_paths(rr_ctx *c)
{
    if (!c->paths_pending) return RR_OK;
    c->paths_pending = false;
    HIPCHK(hipSetDevice(c->device));
    unsigned long long cnt = 0;
    int errf = 0;
    HIPCHK(hipMemcpyAsync(&cnt, c->counter.p, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&errf, c->err_flag.p, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (errf)
        return fail(RR_EUNSUPPORTED, "traversal stack overflow (BVH depth %d)", c->bvh_depth);
    if ((int64_t)cnt > c->tmp_cap) {
        const int64_t need = (int64_t)cnt;
        c->tmp_cap = need + need / 4 + 1024;
        return fail(RR_EOVERFLOW, "%lld paths overflowed the path buffer; it has grown, trace again",
                    (long long)need);
    }
    c->n_paths = std::min<int64_t>((int64_t)cnt, c->pending_keep);
    return RR_OK;
}

}  // namespace

extern "C" {

const char *rr_last_error(void) { return g_err.c_str(); }

const char *rr_version(void) { return "radray 0.1 (gfx950)"; }

int rr_create(int hip_device, void *hip_stream, rr_ctx **out)
{
    if (!out) return fail(RR_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev)
        return fail(RR_EINVAL, "device %d out of range (%d devices)", hip_device, ndev);
    HIPCHK(hipSetDevice(hip_device));
    if (int rc = scratch_init(hip_device)) return rc;
    rr_ctx *c = new rr_ctx();
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    for (auto &e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            rr_destroy(c);
            return fail(RR_EHIP, "hipEventCreate failed");
        }
    }
    int rc = c->counter.ensure(256);
    if (!rc) rc = c->total.ensure(256);
    if (!rc) rc = c->err_flag.ensure(256);
    if (rc) {
        rr_destroy(c);
        return rc;
    }
    *out = c;
    g_err.clear();
    return RR_OK;
}

void rr_destroy(rr_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    DevBuf *bufs[] = {&c->nodes, &c->ltris, &c->obj_alpha, &c->obj_vel, &c->pt_pos, &c->pt_vel,
                      &c->pt_ap, &c->tx, &c->rx, &c->counts, &c->offsets, &c->bsums,
                      &c->counter, &c->total, &c->err_flag, &c->hits, &c->cdf, &c->syn,
                      &c->ranges, &c->tmp.buf, &c->paths.buf, &c->gT, &c->gR, &c->gA,
                      &c->gB, &c->tri_obj, &c->mlp_p, &c->mlp_m, &c->mlp_v, &c->mlp_g,
                      &c->mlp_acts, &c->mlp_z, &c->mlp_dz, &c->mlp_d, &c->mlp_loss, &c->mlp_part,
                      &c->tr_codes, &c->tr_hist, &c->tr_loss, &c->bp_peak, &c->trace_stats, &c->tri_alpha, &c->pieces_v, &c->pieces_p, &c->tris_dev, &c->verts_dev,
                      &c->refit_order, &c->ubox,
                      &c->order_cells, &c->order_rc, &c->order_idx, &c->fq_xt, &c->fq_yt, &c->fq_amp, &c->fq_src, &c->fq_part, &c->bp_sf};
    for (DevBuf *b : bufs) b->release();
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

int rr_scene_upload(rr_ctx *c, const float *verts, int64_t n_verts, const int32_t *tris,
                    const int32_t *tri_obj, int64_t n_tris, const float *obj_alpha,
                    const double *obj_vel, int32_t n_obj, const double *pt_pos,
                    const double *pt_vel, const double *pt_aperture, int32_t n_pts)
{
    if (!c) return fail(RR_EINVAL, "ctx is NULL");
    if (n_verts < 0 || n_tris < 0 || n_obj < 1 || n_pts < 0)
        return fail(RR_EINVAL, "negative size or no object");
    if ((n_tris > 0 && (!verts || !tris || !tri_obj)) || !obj_alpha || !obj_vel ||
        (n_pts > 0 && (!pt_pos || !pt_vel || !pt_aperture)))
        return fail(RR_EINVAL, "NULL array");
    for (int64_t i = 0; i < 3 * n_verts; i++)
        if (!std::isfinite(verts[i])) return fail(RR_EINVAL, "non-finite vertex coordinate");
    for (int64_t i = 0; i < n_tris; i++) {
        for (int k = 0; k < 3; k++)
            if (tris[3 * i + k] < 0 || tris[3 * i + k] >= n_verts)
                return fail(RR_EINVAL, "triangle %lld vertex index out of range", (long long)i);
        if (tri_obj[i] < 0 || tri_obj[i] >= n_obj)
            return fail(RR_EINVAL, "triangle %lld object out of range", (long long)i);
    }
    for (int i = 0; i < n_obj; i++)
        if (!(obj_alpha[i] >= 0.0f && obj_alpha[i] <= 1.0f))
            return fail(RR_EINVAL, "alpha of object %d outside [0, 1]", i);
    if (!finite3(obj_vel, n_obj)) return fail(RR_EINVAL, "non-finite object velocity");
    if (n_pts > 0 && (!finite3(pt_pos, n_pts) || !finite3(pt_vel, n_pts)))
        return fail(RR_EINVAL, "non-finite point reflector");
    for (int i = 0; i < n_pts; i++)
        if (!(pt_aperture[i] >= 0.0) || !std::isfinite(pt_aperture[i]))
            return fail(RR_EINVAL, "invalid point aperture");
    HIPCHK(hipSetDevice(c->device));
    HostBvh bvh;
    std::string err;
    int rc = rr_build_bvh(verts, n_verts, tris, tri_obj, obj_alpha, n_tris, bvh, err);
    if (rc) return fail(rc, "BVH build: %s", err.c_str());
    c->has_scene = false;
    c->n_paths = -1;
    c->paths_pending = false;
    HIPCHK(hipStreamSynchronize(c->stream));
    if ((rc = c->nodes.ensure(bvh.nodes.size() * 4 + 64))) return rc;
    if ((rc = c->ltris.ensure(bvh.tris.size() * 4 + 64))) return rc;
    if ((rc = c->obj_alpha.ensure((size_t)n_obj * 4))) return rc;
    if ((rc = c->obj_vel.ensure((size_t)n_obj * 24))) return rc;
    if ((rc = c->pt_pos.ensure((size_t)n_pts * 24 + 8))) return rc;
    if ((rc = c->pt_vel.ensure((size_t)n_pts * 24 + 8))) return rc;
    if ((rc = c->pt_ap.ensure((size_t)n_pts * 8 + 8))) return rc;
    if ((rc = c->tri_obj.ensure((size_t)n_tris * 4 + 8))) return rc;
    if (n_tris > 0)
        HIPCHK(hipMemcpy(c->tri_obj.p, tri_obj, (size_t)n_tris * 4, hipMemcpyHostToDevice));
    c->h_verts.assign(verts, verts + 3 * n_verts);
    c->pieces_valid = false;
    if (!bvh.nodes.empty())
        HIPCHK(hipMemcpy(c->nodes.p, bvh.nodes.data(), bvh.nodes.size() * 4, hipMemcpyHostToDevice));
    if (!bvh.tris.empty())
        HIPCHK(hipMemcpy(c->ltris.p, bvh.tris.data(), bvh.tris.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->obj_alpha.p, obj_alpha, (size_t)n_obj * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->obj_vel.p, obj_vel, (size_t)n_obj * 24, hipMemcpyHostToDevice));
    if (n_pts > 0) {
        HIPCHK(hipMemcpy(c->pt_pos.p, pt_pos, (size_t)n_pts * 24, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->pt_vel.p, pt_vel, (size_t)n_pts * 24, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->pt_ap.p, pt_aperture, (size_t)n_pts * 8, hipMemcpyHostToDevice));
    }
    // refit support: topology on the device, internal nodes by depth (deepest first)
    c->refit_levels.clear();
    c->n_nodes = (int64_t)bvh.nodes.size() / 16;
    if (n_tris > 0) {
        std::vector<std::vector<int32_t>> lv;
        std::vector<int32_t> cur{0};
        while (!cur.empty()) {
            lv.push_back(cur);
            std::vector<int32_t> nxt;
            for (int32_t n : cur)
                for (int ch = 0; ch < 2; ch++) {
                    int32_t ref;
                    std::memcpy(&ref, &bvh.nodes[16 * (size_t)n + 12 + ch], 4);
                    if (ref >= 0) nxt.push_back(ref);
                }
            cur.swap(nxt);
        }
        std::vector<int32_t> order;
        for (size_t l = lv.size(); l-- > 0;) {
            c->refit_levels.push_back((int64_t)order.size());
            order.insert(order.end(), lv[l].begin(), lv[l].end());
        }
        c->refit_levels.push_back((int64_t)order.size());
        if ((rc = c->refit_order.ensure(order.size() * 4 + 8))) return rc;
        if ((rc = c->ubox.ensure((size_t)c->n_nodes * 24 + 8))) return rc;
        if ((rc = c->tris_dev.ensure((size_t)n_tris * 12))) return rc;
        if ((rc = c->verts_dev.ensure((size_t)n_verts * 12 + 8))) return rc;
        HIPCHK(hipMemcpy(c->refit_order.p, order.data(), order.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->tris_dev.p, tris, (size_t)n_tris * 12, hipMemcpyHostToDevice));
        c->h_tris.assign(tris, tris + 3 * n_tris);
    } else {
        c->h_tris.clear();
    }
    c->n_verts = n_verts;
    c->n_tris = n_tris;
    c->nobj = n_obj;
    c->npts = n_pts;
    c->bvh_depth = bvh.depth;
    c->has_scene = true;
    g_err.clear();
    return RR_OK;
}

int rr_scene_update_vertices(rr_ctx *c, const float *verts, int64_t n_verts)
{
    if (!c) return fail(RR_EINVAL, "ctx is NULL");
    if (!c->has_scene) return fail(RR_ESTATE, "no scene uploaded");
    if (n_verts != c->n_verts)
        return fail(RR_EINVAL, "vertex count %lld differs from the uploaded scene's %lld",
                    (long long)n_verts, (long long)c->n_verts);
    if (n_verts > 0 && !verts) return fail(RR_EINVAL, "NULL vertices");
    for (int64_t i = 0; i < 3 * n_verts; i++)
        if (!std::isfinite(verts[i])) return fail(RR_EINVAL, "non-finite vertex coordinate");
    if (c->n_tris == 0) return RR_OK;
    // the padding of the host build, from the vertices the triangles use
    double maxabs = 0.0;
    for (int64_t i = 0; i < 3 * c->n_tris; i++) {
        const float *v = verts + 3 * (int64_t)c->h_tris[i];
        for (int a = 0; a < 3; a++) maxabs = std::max(maxabs, (double)std::fabs(v[a]));
    }
    const double pad = 1e-3 + 1e-6 * maxabs;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(c->verts_dev.p, verts, (size_t)n_verts * 12, hipMemcpyHostToDevice));
    HIPCHK(launch_refit(c->nodes.as<float4>(), c->ubox.as<float>(), c->refit_order.as<const int32_t>(),
                        c->refit_levels.data(), (int)c->refit_levels.size() - 1, c->ltris.as<float4>(),
                        c->n_tris, c->tris_dev.as<const int32_t>(), c->verts_dev.as<const float>(),
                        pad, c->stream));
    c->h_verts.assign(verts, verts + 3 * n_verts);
    c->pieces_valid = false;
    g_err.clear();
    return RR_OK;
}

int rr_get_bvh_nodes(rr_ctx *c, float *dst, int64_t capacity, int64_t *n_floats)
{
    if (!c || !n_floats) return fail(RR_EINVAL, "NULL argument");
    if (!c->has_scene) return fail(RR_ESTATE, "no scene uploaded");
    *n_floats = 16 * c->n_nodes;
    if (!dst) return RR_OK;
    if (capacity < *n_floats) return fail(RR_EOVERFLOW, "need %lld floats", (long long)*n_floats);
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (*n_floats > 0)
        HIPCHK(hipMemcpy(dst, c->nodes.p, (size_t)*n_floats * 4, hipMemcpyDeviceToHost));
    g_err.clear();
    return RR_OK;
}

namespace {

// Replace the material mix of a scene's leaf records: alpha[n] per face
// (n = n_tris, by upload index) or per object (n = n_obj).  The stream is
// drained first so that no earlier launch still reads the staging buffers.
int set_alpha_common(hipStream_t st, DevBuf &ltris, DevBuf &obj_buf, DevBuf &tri_buf,
                     int64_t n_tris, int nobj, const float *alpha, int64_t n, int32_t per)
{
    if (!alpha && n > 0) return fail(RR_EINVAL, "NULL alpha");
    if (per == RR_ALPHA_PER_OBJECT) {
        if (n != nobj) return fail(RR_EINVAL, "per-object alpha needs one value per object (%d)", nobj);
    } else if (per == RR_ALPHA_PER_TRIANGLE) {
        if (n != n_tris)
            return fail(RR_EINVAL, "per-face alpha needs one value per triangle (%lld)", (long long)n_tris);
    } else {
        return fail(RR_EINVAL, "unknown alpha mode");
    }
    for (int64_t i = 0; i < n; i++)
        if (!(alpha[i] >= 0.0f && alpha[i] <= 1.0f))
            return fail(RR_EINVAL, "alpha %lld outside [0, 1]", (long long)i);
    HIPCHK(hipStreamSynchronize(st));
    int rc;
    if (per == RR_ALPHA_PER_OBJECT) {
        HIPCHK(hipMemcpy(obj_buf.p, alpha, (size_t)n * 4, hipMemcpyHostToDevice));
        HIPCHK(launch_set_alpha(ltris.as<float4>(), n_tris, nullptr, obj_buf.as<const float>(), st));
    } else if (n > 0) {
        if ((rc = tri_buf.ensure((size_t)n * 4))) return rc;
        HIPCHK(hipMemcpy(tri_buf.p, alpha, (size_t)n * 4, hipMemcpyHostToDevice));
        HIPCHK(launch_set_alpha(ltris.as<float4>(), n_tris, tri_buf.as<const float>(), nullptr, st));
    }
    return RR_OK;
}

}  // namespace

int rr_scene_set_alpha(rr_ctx *c, const float *alpha, int64_t n, int32_t per)
{
    if (!c) return fail(RR_EINVAL, "ctx is NULL");
    if (!c->has_scene) return fail(RR_ESTATE, "no scene uploaded");
    HIPCHK(hipSetDevice(c->device));
    int rc = set_alpha_common(c->stream, c->ltris, c->obj_alpha, c->tri_alpha, c->n_tris, c->nobj,
                              alpha, n, per);
    if (rc) return rc;
    g_err.clear();
    return RR_OK;
}

namespace {

// the per-triangle launch's pieces for the current scene, array, casting
// parameters and field of view (rebuilt when any of them changed)
int ensure_pieces(rr_ctx *c, const rr_trace_params *tp)
{
    const double fov[4] = {tp->az_min, tp->az_max, tp->el_min, tp->el_max};
    if (c->pieces_valid && std::equal(fov, fov + 4, c->cast_fov)) return RR_OK;
    RrFov f;
    const int shared = c->mode == RR_TX_SHARED;
    f.src = shared ? c->oT : c->h_tx.data();
    f.n_src = shared ? 1 : c->ntx;
    f.c0 = std::cos(tp->az_min);
    f.s0 = std::sin(tp->az_min);
    f.c1 = std::cos(tp->az_max);
    f.s1 = std::sin(tp->az_max);
    f.slo = std::sin(tp->el_min);
    f.shi = std::sin(tp->el_max);
    std::vector<double> pv;
    std::vector<int32_t> par;
    const int64_t limit = (int64_t)1 << 26;
    int rc = rr_build_pieces(c->h_verts.data(), c->h_tris.data(), c->n_tris, c->oT, c->cast_omega,
                             c->cast_depth, &f, limit, pv, par);
    if (rc) return fail(rc, "more than %lld pieces: raise the solid-angle limit", (long long)limit);
    HIPCHK(hipStreamSynchronize(c->stream));
    if ((rc = c->pieces_v.ensure(pv.size() * 8 + 8))) return rc;
    if ((rc = c->pieces_p.ensure(par.size() * 4 + 8))) return rc;
    if (!par.empty()) {
        HIPCHK(hipMemcpy(c->pieces_v.p, pv.data(), pv.size() * 8, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->pieces_p.p, par.data(), par.size() * 4, hipMemcpyHostToDevice));
    }
    c->n_pieces = (int64_t)par.size();
    std::copy(fov, fov + 4, c->cast_fov);
    c->pieces_valid = true;
    return RR_OK;
}

}  // namespace

int rr_set_casting(rr_ctx *c, double max_solid_angle, int32_t max_depth)
{
    if (!c) return fail(RR_EINVAL, "ctx is NULL");
    if (!(max_solid_angle >= 0.0) || !std::isfinite(max_solid_angle) || max_depth < 0 ||
        max_depth > 20)
        return fail(RR_EINVAL, "need max_solid_angle >= 0 and 0 <= max_depth <= 20");
    if (c->cast_omega != max_solid_angle || c->cast_depth != max_depth) c->pieces_valid = false;
    c->cast_omega = max_solid_angle;
    c->cast_depth = max_depth;
    g_err.clear();
    return RR_OK;
}

int rr_casting_pieces(rr_ctx *c, const rr_trace_params *tp, int64_t *n_pieces)
{
    if (!c || !tp || !n_pieces) return fail(RR_EINVAL, "NULL argument");
    if (!c->has_scene || !c->has_array) return fail(RR_ESTATE, "scene and array must be set");
    if (!(tp->az_max > tp->az_min) || !(tp->az_max - tp->az_min <= M_PI) ||
        !(tp->el_max > tp->el_min) || !std::isfinite(tp->az_min) || !std::isfinite(tp->el_min))
        return fail(RR_EINVAL, "invalid field of view for per-triangle casting");
    HIPCHK(hipSetDevice(c->device));
    int rc = ensure_pieces(c, tp);
    if (rc) return rc;
    *n_pieces = c->n_pieces;
    g_err.clear();
    return RR_OK;
}

int rr_set_array(rr_ctx *c, const double *tx, int32_t n_tx, const double *rx, int32_t n_rx,
                 double rx_radius, int32_t tx_mode)
{
    if (!c) return fail(RR_EINVAL, "ctx is NULL");
    if (!tx || !rx || n_tx < 1 || n_rx < 1) return fail(RR_EINVAL, "empty array");
    if (!finite3(tx, n_tx) || !finite3(rx, n_rx)) return fail(RR_EINVAL, "non-finite element");
    if (!(rx_radius > 0.0) || !std::isfinite(rx_radius))
        return fail(RR_EINVAL, "rx_radius must be positive");
    if (tx_mode != RR_TX_PER_ELEMENT && tx_mode != RR_TX_SHARED)
        return fail(RR_EINVAL, "unknown tx_mode %d", tx_mode);
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    int rc;
    if ((rc = c->tx.ensure((size_t)n_tx * 24))) return rc;
    if ((rc = c->rx.ensure((size_t)n_rx * 24))) return rc;
    HIPCHK(hipMemcpy(c->tx.p, tx, (size_t)n_tx * 24, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->rx.p, rx, (size_t)n_rx * 24, hipMemcpyHostToDevice));
    c->pieces_valid = false;
    c->h_tx.assign(tx, tx + 3 * n_tx);
    c->h_rx.assign(rx, rx + 3 * n_rx);
    c->tx_h.assign(tx, tx + 3 * n_tx);
    c->rx_h.assign(rx, rx + 3 * n_rx);
    // phase centres: sums in index order divided by the count
    for (int a = 0; a < 3; a++) {
        double s = 0.0;
        for (int i = 0; i < n_tx; i++) s += tx[3 * i + a];
        c->oT[a] = s / (double)n_tx;
        s = 0.0;
        for (int i = 0; i < n_rx; i++) s += rx[3 * i + a];
        c->oR[a] = s / (double)n_rx;
    }
    c->ntx = n_tx;
    c->nrx = n_rx;
    c->rx_radius = rx_radius;
    c->mode = tx_mode;
    c->has_array = true;
    c->n_paths = -1;
    c->paths_pending = false;
    g_err.clear();
    return RR_OK;
}

int rr_set_chirp(rr_ctx *c, const rr_chirp *ch)
{
    if (!c || !ch) return fail(RR_EINVAL, "NULL argument");
    if (!(ch->f0 > 0.0) || !std::isfinite(ch->f0) || !(ch->bandwidth >= 0.0) ||
        !std::isfinite(ch->bandwidth) || !(ch->t_chirp > 0.0) || !(ch->t_rep >= 0.0) ||
        !std::isfinite(ch->t_rep) || ch->n_samples < 1 || ch->n_chirps < 1)
        return fail(RR_EINVAL, "degenerate chirp");
    c->chirp = *ch;
    c->has_chirp = true;
    g_err.clear();
    return RR_OK;
}

// defined below; also used by the proposal code
int rr_set_proposal_cdf_internal(rr_ctx *c, const double *cdf_dev, int n_az, int n_el);

// rr_trace, with the counting kernel when stats (device, 3 x u64) is given
static int trace_impl(rr_ctx *c, const rr_trace_params *tp, int64_t *n_paths_out,
                      unsigned long long *stats)
{
    if (!c || !tp) return fail(RR_EINVAL, "NULL argument");
    if (!c->has_scene || !c->has_array) return fail(RR_ESTATE, "scene and array must be set");
    if (tp->max_bounces < 1 || tp->max_bounces > RR_KMAX)
        return fail(RR_EINVAL, "max_bounces must be in [1, %d]", RR_KMAX);
    if (tp->n_rays < 0) return fail(RR_EINVAL, "negative n_rays");
    if (!(tp->az_max > tp->az_min) || !(tp->el_max > tp->el_min) || tp->el_min < -M_PI / 2 - 1e-12 ||
        tp->el_max > M_PI / 2 + 1e-12 || !std::isfinite(tp->az_min) || !std::isfinite(tp->az_max))
        return fail(RR_EINVAL, "invalid field of view");
    if (tp->sampler != RR_UNIFORM && tp->sampler != RR_PROPOSAL && tp->sampler != RR_PER_TRIANGLE)
        return fail(RR_EINVAL, "unknown sampler");
    int tri_g = 0;
    if (tp->sampler == RR_PER_TRIANGLE) {
        tri_g = (int)std::llround(std::sqrt((double)tp->n_rays));
        if (tp->n_rays < 1 || (int64_t)tri_g * tri_g != tp->n_rays)
            return fail(RR_EINVAL, "per-triangle casting needs n_rays = g^2 >= 1 rays per triangle");
        if (!(tp->az_max - tp->az_min <= M_PI))
            return fail(RR_EINVAL, "per-triangle casting needs an azimuth span of at most pi");
    }
    if (tp->sampler == RR_PROPOSAL && c->n_az <= 0)
        return fail(RR_ESTATE, "proposal sampler without a proposal table");
    if (tp->path_cap < 0) return fail(RR_EINVAL, "negative path_cap");
    HIPCHK(hipSetDevice(c->device));

    const int shared = c->mode == RR_TX_SHARED;
    const int64_t n_src = shared ? 1 : c->ntx;
    if (tri_g) {
        const int rp = ensure_pieces(c, tp);
        if (rp) return rp;
    }
    const int64_t n_per_src = tri_g ? c->n_pieces * tp->n_rays
                                    : shared ? tp->n_rays : tp->n_rays / c->ntx;
    const int64_t n_vps = n_per_src + c->npts;
    const int64_t V = n_src * n_vps;
    const int64_t n_traced = n_src * n_per_src;
    if (V >= (int64_t(1) << 32)) return fail(RR_EUNSUPPORTED, "too many rays");
    const int bmax = tp->max_bounces;

    int rc;
    if ((rc = c->counts.ensure((size_t)V + 64))) return rc;
    if ((rc = c->offsets.ensure((size_t)V * 4 + 64))) return rc;
    const int64_t nb = scan_u8_blocks(V);
    if ((rc = c->bsums.ensure((size_t)(nb + 1) * 4))) return rc;
    if (tp->record_hits) {
        if ((rc = c->hits.ensure((size_t)n_traced * (bmax + 1) * 4 + 64))) return rc;
        c->hits_elems = n_traced * (bmax + 1);
        c->hits_recorded = true;
    } else {
        c->hits_elems = 0;
        c->hits_recorded = false;
    }
    if (c->tmp_cap == 0) c->tmp_cap = std::max<int64_t>(65536, V / 32);
    if ((rc = c->tmp.alloc(c->tmp_cap))) return rc;
    // uniform and proposal launches trace their rays in a coherent order
    // (sorted by source and first-direction cell; results do not depend on it)
    const bool coherent = !tri_g && n_per_src >= 4096 && n_traced < ((int64_t)1 << 31);
    const int obits = coherent ? trace_order_bits(n_per_src) : 0;
    if (coherent) {
        if ((rc = c->order_idx.ensure((size_t)n_traced * 4))) return rc;
        if ((rc = c->order_rc.ensure((size_t)n_traced * 2))) return rc;
        if ((rc = c->order_cells.ensure((size_t)(n_src << (2 * obits)) * 4))) return rc;
    }

    TraceArgs A{};
    A.nodes = c->nodes.as<const float4>();
    A.ltris = c->ltris.as<const float4>();
    A.has_bvh = c->n_tris > 0;
    A.tx = c->tx.as<const double>();
    A.pt_pos = c->pt_pos.as<const double>();
    A.pt_ap = c->pt_ap.as<const double>();
    for (int a = 0; a < 3; a++) {
        A.oT[a] = c->oT[a];
        A.oR[a] = c->oR[a];
    }
    A.r2 = c->rx_radius * c->rx_radius;
    A.shared = shared;
    A.nobj = c->nobj;
    A.npts = c->npts;
    A.n_src = n_src;
    A.n_per_src = n_per_src;
    A.n_virt_per_src = n_vps;
    const double INV_2PI = 0.15915494309189535;
    A.at = tp->az_min * INV_2PI;
    A.bt = tp->az_max * INV_2PI;
    A.slo = std::sin(tp->el_min);
    A.shi = std::sin(tp->el_max);
    A.omega = (tp->az_max - tp->az_min) * (A.shi - A.slo);
    A.bmax = bmax;
    A.seed = tp->seed;
    A.sampler = tp->sampler;
    A.cdf = c->cdf.as<const double>();
    A.n_az = c->n_az;
    A.n_el = c->n_el;
    A.pieces = c->pieces_v.as<const double>();
    A.piece_parent = c->pieces_p.as<const int32_t>();
    A.tri_g = tri_g;
    A.fov_c0 = std::cos(tp->az_min);
    A.fov_s0 = std::sin(tp->az_min);
    A.fov_c1 = std::cos(tp->az_max);
    A.fov_s1 = std::sin(tp->az_max);
    A.hits = tp->record_hits ? c->hits.as<int32_t>() : nullptr;
    A.counts = c->counts.as<uint8_t>();
    A.counter = c->counter.as<unsigned long long>();
    A.err_flag = c->err_flag.as<int>();

    auto kernels = [&](const TraceArgs &a) -> hipError_t {
        hipError_t e = hipSuccess;
        TraceArgs b = a;
        if (coherent) {
            e = launch_trace_order(a, n_traced, obits, c->order_cells.as<unsigned>(),
                                   c->order_rc.as<uint16_t>(), c->order_idx.as<int32_t>(),
                                   c->stream);
            b.order = c->order_idx.as<const int32_t>();
        }
        if (e == hipSuccess && stats) {
            e = hipMemsetAsync(stats, 0, 3 * sizeof(unsigned long long), c->stream);
            if (e == hipSuccess) e = launch_trace_count(b, n_traced, stats, c->stream);
        } else if (e == hipSuccess) {
            e = launch_trace(b, n_traced, c->stream);
        }
        return e == hipSuccess ? launch_points(a, c->stream) : e;
    };
    int rc2 = run_trace(c, A, V, nb, tp->path_cap, kernels, n_paths_out);
    if (rc2) return rc2;
    c->last_traced = n_traced;
    c->last_sampler = tp->record_hits ? tp->sampler : -1;
    return RR_OK;
}

int rr_trace(rr_ctx *c, const rr_trace_params *tp, int64_t *n_paths_out)
{
    return trace_impl(c, tp, n_paths_out, nullptr);
}

int rr_trace_work(rr_ctx *c, const rr_trace_params *tp, int64_t *n_paths_out, int64_t work_out[4])
{
    if (!c || !tp || !n_paths_out || !work_out) return fail(RR_EINVAL, "NULL argument");
    if (!c->has_scene || !c->has_array) return fail(RR_ESTATE, "scene and array must be set");
    HIPCHK(hipSetDevice(c->device));
    int rc = c->trace_stats.ensure(64);
    if (rc) return rc;
    if ((rc = trace_impl(c, tp, n_paths_out, c->trace_stats.as<unsigned long long>()))) return rc;
    unsigned long long st[3] = {0, 0, 0};
    HIPCHK(hipMemcpyAsync(st, c->trace_stats.p, sizeof(st), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    work_out[0] = c->last_traced;
    work_out[1] = (int64_t)st[2];
    work_out[2] = (int64_t)st[0];
    work_out[3] = (int64_t)st[1];
    return RR_OK;
}

// Caller-supplied rays: validated on the device, then traced like the launch.
int rr_trace_rays(rr_ctx *c, const double *orig, const double *dir, const double *amp,
                  const int32_t *src, int64_t n, int32_t max_bounces, uint64_t seed,
                  int32_t record_hits, int64_t *n_paths_out)
{
    if (!c) return fail(RR_EINVAL, "NULL argument");
    if (!c->has_scene || !c->has_array) return fail(RR_ESTATE, "scene and array must be set");
    if (max_bounces < 1 || max_bounces > RR_KMAX)
        return fail(RR_EINVAL, "max_bounces must be in [1, %d]", RR_KMAX);
    if (n < 0) return fail(RR_EINVAL, "negative ray count");
    if (n > 0 && (!orig || !dir || !amp || !src)) return fail(RR_EINVAL, "NULL ray array");
    if (n >= (int64_t(1) << 32)) return fail(RR_EUNSUPPORTED, "too many rays");
    HIPCHK(hipSetDevice(c->device));
    const int shared = c->mode == RR_TX_SHARED;
    UserRays U{orig, dir, amp, src, n};
    int rc;
    if (n > 0) {
        int bad = 0;
        HIPCHK(hipMemsetAsync(c->err_flag.p, 0, 4, c->stream));
        HIPCHK(launch_check_user(U, shared, c->ntx, c->err_flag.as<int>(), c->stream));
        HIPCHK(hipMemcpyAsync(&bad, c->err_flag.p, 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (bad)
            return fail(RR_EINVAL, shared ? "rays: sources must be -1 (shared launch), vectors finite, directions non-zero"
                                          : "rays: sources must ascend within [0, n_tx), vectors finite, directions non-zero");
    }
    const int64_t V = n;
    if ((rc = c->counts.ensure((size_t)V + 64))) return rc;
    if ((rc = c->offsets.ensure((size_t)V * 4 + 64))) return rc;
    const int64_t nb = scan_u8_blocks(V);
    if ((rc = c->bsums.ensure((size_t)(nb + 1) * 4))) return rc;
    if (record_hits) {
        if ((rc = c->hits.ensure((size_t)n * (max_bounces + 1) * 4 + 64))) return rc;
        c->hits_elems = n * (max_bounces + 1);
        c->hits_recorded = true;
    } else {
        c->hits_elems = 0;
        c->hits_recorded = false;
    }
    if (c->tmp_cap == 0) c->tmp_cap = std::max<int64_t>(65536, V / 32);
    if ((rc = c->tmp.alloc(c->tmp_cap))) return rc;

    TraceArgs A{};
    A.nodes = c->nodes.as<const float4>();
    A.ltris = c->ltris.as<const float4>();
    A.has_bvh = c->n_tris > 0;
    A.tx = c->tx.as<const double>();
    for (int a = 0; a < 3; a++) {
        A.oT[a] = c->oT[a];
        A.oR[a] = c->oR[a];
    }
    A.r2 = c->rx_radius * c->rx_radius;
    A.shared = shared;
    A.nobj = c->nobj;
    A.npts = 0;
    A.n_src = 1;
    A.n_per_src = n;
    A.n_virt_per_src = n;
    A.bmax = max_bounces;
    A.seed = seed;
    A.sampler = RR_UNIFORM;
    A.hits = record_hits ? c->hits.as<int32_t>() : nullptr;
    A.counts = c->counts.as<uint8_t>();
    A.counter = c->counter.as<unsigned long long>();
    A.err_flag = c->err_flag.as<int>();
    auto kernels = [&](const TraceArgs &a) -> hipError_t {
        return launch_trace_user(a, U, c->stream);
    };
    if ((rc = run_trace(c, A, V, nb, 0, kernels, n_paths_out))) return rc;
    c->last_traced = n;
    c->last_sampler = -1;
    return RR_OK;
}



int rr_get_path_count(rr_ctx *c, int64_t *n_out)
{
    if (!c || !n_out) return fail(RR_EINVAL, "NULL argument");
    if (int rc = resolve_paths(c)) return rc;
    if (c->n_paths < 0) return fail(RR_ESTATE, "no paths");
    *n_out = c->n_paths;
    return RR_OK;
}

int rr_get_hits(rr_ctx *c, int32_t *dst, int64_t cap_elems)
{
    if (!c) return fail(RR_EINVAL, "NULL argument");
    if (int rc = resolve_paths(c)) return rc;
    if (c->n_paths < 0 || !c->hits_recorded) return fail(RR_ESTATE, "no hit list recorded");
    if (c->hits_elems == 0) return RR_OK;
    if (!dst) return fail(RR_EINVAL, "NULL argument");
    if (cap_elems < c->hits_elems)
        return fail(RR_EOVERFLOW, "hit list needs %lld elements", (long long)c->hits_elems);
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipMemcpyAsync(dst, c->hits.p, (size_t)c->hits_elems * 4, hipMemcpyDeviceToDevice,
                          c->stream));
    return RR_OK;
}

static hipError_t copy_planes(void *dst, int64_t dstride, const void *src, int64_t sstride,
                              int64_t n, int planes, size_t esz, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    return hipMemcpy2DAsync(dst, (size_t)dstride * esz, src, (size_t)sstride * esz, (size_t)n * esz,
                            (size_t)planes, hipMemcpyDeviceToDevice, s);
}

int rr_get_paths(rr_ctx *c, const rr_paths *d, int64_t *n_out)
{
    if (!c || !d || !n_out) return fail(RR_EINVAL, "NULL argument");
    if (int rc = resolve_paths(c)) return rc;
    if (c->n_paths < 0) return fail(RR_ESTATE, "no paths");
    int64_t n = c->n_paths;
    *n_out = n;
    if (d->stride < n) return fail(RR_EOVERFLOW, "need capacity %lld", (long long)n);
    HIPCHK(hipSetDevice(c->device));
    const PathSoA &s = c->paths.soa;
    hipStream_t st = c->stream;
    if (d->src) HIPCHK(copy_planes(d->src, d->stride, s.src, s.cap, n, 1, 4, st));
    if (d->K) HIPCHK(copy_planes(d->K, d->stride, s.K, s.cap, n, 1, 4, st));
    if (d->ray) HIPCHK(copy_planes(d->ray, d->stride, s.ray, s.cap, n, 1, 8, st));
    if (d->tri) HIPCHK(copy_planes(d->tri, d->stride, s.tri, s.cap, n, RR_KMAX, 4, st));
    if (d->vid) HIPCHK(copy_planes(d->vid, d->stride, s.vid, s.cap, n, RR_KMAX, 4, st));
    if (d->p) HIPCHK(copy_planes(d->p, d->stride, s.p, s.cap, n, 3 * RR_KMAX, 8, st));
    if (d->L) HIPCHK(copy_planes(d->L, d->stride, s.L, s.cap, n, 1, 8, st));
    if (d->amp) HIPCHK(copy_planes(d->amp, d->stride, s.amp, s.cap, n, 1, 8, st));
    HIPCHK(hipStreamSynchronize(st));
    return RR_OK;
}

int rr_set_paths(rr_ctx *c, const rr_paths *s, int64_t n)
{
    if (!c || !s) return fail(RR_EINVAL, "NULL argument");
    if (n < 0 || s->stride < n) return fail(RR_EINVAL, "bad count or stride");
    if (n > 0 && (!s->src || !s->K || !s->vid || !s->p || !s->amp))
        return fail(RR_EINVAL, "src, K, vid, p and amp are required");
    HIPCHK(hipSetDevice(c->device));
    c->paths_pending = false;
    int rc = c->paths.alloc(std::max<int64_t>(n, 1));
    if (rc) return rc;
    const PathSoA &d = c->paths.soa;
    hipStream_t st = c->stream;
    HIPCHK(copy_planes(d.src, d.cap, s->src, s->stride, n, 1, 4, st));
    HIPCHK(copy_planes(d.K, d.cap, s->K, s->stride, n, 1, 4, st));
    HIPCHK(copy_planes(d.vid, d.cap, s->vid, s->stride, n, RR_KMAX, 4, st));
    HIPCHK(copy_planes(d.p, d.cap, s->p, s->stride, n, 3 * RR_KMAX, 8, st));
    HIPCHK(copy_planes(d.amp, d.cap, s->amp, s->stride, n, 1, 8, st));
    if (s->ray) HIPCHK(copy_planes(d.ray, d.cap, s->ray, s->stride, n, 1, 8, st));
    if (s->tri) HIPCHK(copy_planes(d.tri, d.cap, s->tri, s->stride, n, RR_KMAX, 4, st));
    if (s->L) HIPCHK(copy_planes(d.L, d.cap, s->L, s->stride, n, 1, 8, st));
    // validate on the host: K in range, src sorted and in range
    std::vector<int32_t> hs(n), hk(n);
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(hs.data(), d.src, n * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hk.data(), d.K, n * 4, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n; i++) {
        if (hk[i] < 1 || hk[i] > RR_KMAX) {
            c->n_paths = -1;
            return fail(RR_EINVAL, "path %lld: K out of range", (long long)i);
        }
        if (hs[i] < -1 || (i > 0 && hs[i] < hs[i - 1])) {
            c->n_paths = -1;
            return fail(RR_EINVAL, "path %lld: src must be >= -1 and sorted", (long long)i);
        }
    }
    c->n_paths = n;
    g_err.clear();
    return RR_OK;
}

// separable model on the matrix cores: operand preparation, then the GEMM
// (the context's events bracket the GEMM kernel alone)
static int rr_synth_gemm(rr_ctx *c, const SynthArgs &A)
{
    const int C = c->ntx * c->nrx;
    const int Cpad = (C + gemm_row_pad() - 1) / gemm_row_pad() * gemm_row_pad();
    const int64_t n = A.n_paths;
    const int ks = gemm_k_step();
    const int64_t Ppad = std::max<int64_t>((n + ks - 1) / ks * ks, ks);
    if (Ppad > (int64_t)1 << 30) return fail(RR_EUNSUPPORTED, "too many paths for the GEMM engine");
    int rc;
    if ((rc = c->gT.ensure((size_t)c->ntx * Ppad * 8))) return rc;
    if ((rc = c->gR.ensure((size_t)c->nrx * Ppad * 8))) return rc;
    if ((rc = c->gA.ensure((size_t)Cpad * Ppad * gemm_a_bytes()))) return rc;
    if ((rc = c->gB.ensure((size_t)A.M * Ppad * 16))) return rc;
    HIPCHK(launch_gemm_prep_tr(A, (int)Ppad, c->gT.as<float2>(), c->gR.as<float2>(), c->stream));
    HIPCHK(launch_gemm_prep_a(c->gT.as<const float2>(), c->gR.as<const float2>(), c->nrx, C, Cpad,
                              (int)Ppad, c->gA.as<uint4>(), c->stream));
    HIPCHK(launch_gemm_prep_b(A, (int)Ppad, c->gB.as<uint4>(), c->stream));
    HIPCHK(hipEventRecord(c->ev[2], c->stream));
    HIPCHK(launch_gemm_main(c->gA.as<const uint4>(), c->gB.as<const uint4>(), Cpad, (int)Ppad, C,
                            A.M, A.K, A.cube, c->stream));
    return RR_OK;
}

// Exact model as one complex product per (chirp, sample): leg tables per
// (chirp, element, path), then the split-bf16 MFMA kernel over path splits.
static const int64_t FREQ_TABLE_MAX = (int64_t)16 << 30;   // AUTO's table budget (bytes)

static int64_t freq_table_bytes(const rr_ctx *c, int64_t n)
{
    const int64_t ks = freq_k_step();
    const int64_t Ppad = std::max<int64_t>((n + ks - 1) / ks * ks, ks);
    const bool per_el = c->mode != RR_TX_SHARED;
    const bool own = freq_own_tx(freq_tile(c->ntx, c->nrx, c->chirp.n_samples, per_el), per_el, true);
    return 8 * freq_table_entries(c->ntx, c->nrx, c->chirp.n_chirps, Ppad, own);
}

static int rr_synth_freq(rr_ctx *c, const SynthArgs &A)
{
    const int64_t n = A.n_paths;
    const int64_t ks = freq_k_step();
    const int64_t Ppad = std::max<int64_t>((n + ks - 1) / ks * ks, ks);
    const int T = c->ntx, R = c->nrx, M = A.M, K = A.K;
    const bool per_el = c->mode != RR_TX_SHARED;
    const int tile = freq_tile(T, R, K, per_el);
    int n_split = 1;
    int64_t split_len = Ppad;
    freq_splits(tile, T, R, M, K, Ppad, n_split, split_len);
    const bool own = freq_own_tx(tile, per_el, A.ranges != nullptr);
    int rc;
    if ((rc = c->fq_xt.ensure((size_t)M * (own ? 1 : T) * Ppad * 8))) return rc;
    if ((rc = c->fq_yt.ensure((size_t)M * R * Ppad * 8))) return rc;
    if ((rc = c->fq_amp.ensure((size_t)Ppad * 4))) return rc;
    if ((rc = c->fq_src.ensure((size_t)Ppad * 4))) return rc;
    if (n_split > 1 && (rc = c->fq_part.ensure((size_t)n_split * M * K * T * R * 8))) return rc;
    HIPCHK(hipEventRecord(c->ev[2], c->stream));
    HIPCHK(launch_freq_prep(A.paths, n, nullptr, nullptr, Ppad, M, A.t_rep, A.tx, T, own, A.rx, R,
                            A.f0 * A.inv_c, A.bw / (double)K * A.inv_c, c->fq_xt.as<uint2>(),
                            c->fq_yt.as<uint2>(), c->fq_amp.as<float>(), c->fq_src.as<int32_t>(),
                            c->stream));
    HIPCHK(launch_freq_gemm(c->fq_xt.as<const uint2>(), c->fq_yt.as<const uint2>(),
                            c->fq_amp.as<const float>(), c->fq_src.as<const int32_t>(), T, R, M, K,
                            Ppad, (int)n_split, split_len, per_el, tile, nullptr, nullptr,
                            per_el ? A.ranges : nullptr, c->fq_part.as<float2>(), A.cube,
                            c->stream));
    return RR_OK;
}

int rr_synthesize(rr_ctx *c, int32_t model, int32_t engine, void *cube, int64_t cube_elems,
                  const int64_t *idx, int64_t n_idx)
{
    if (!c || !cube) return fail(RR_EINVAL, "NULL argument");
    if (!c->has_array || !c->has_chirp) return fail(RR_ESTATE, "array and chirp must be set");
    if (int rc = resolve_paths(c)) return rc;
    if (c->n_paths < 0) return fail(RR_ESTATE, "no paths (trace or rr_set_paths first)");
    if (model != RR_EXACT && model != RR_SEPARABLE) return fail(RR_EINVAL, "unknown model");
    if (engine == RR_ENGINE_AUTO) {
        // the GEMM engine pads each chirp's samples to whole column tiles:
        // take it for the separable model when that pads by at most a quarter
        const int64_t K = c->chirp.n_samples, CT = gemm_col_tile();
        const int64_t Kp = (K + CT - 1) / CT * CT;
        engine = (model == RR_SEPARABLE && !idx && 4 * Kp <= 5 * K) ? RR_GEMM_BF16X3
                                                                     : RR_DIRECT_FP32;
        // the exact model as products on the matrix cores: where the best
        // product layout is modelled at least 1.5x the direct engine's
        // throughput and the leg tables fit the budget
        if (model == RR_EXACT && !idx && c->n_paths > 0 &&
            freq_pays(c->ntx, c->nrx, (int)K, c->mode != RR_TX_SHARED) &&
            freq_table_bytes(c, c->n_paths) <= FREQ_TABLE_MAX)
            engine = RR_GEMM_EXACT;
    }
    if (engine != RR_DIRECT_FP32 && engine != RR_GEMM_BF16X3 && engine != RR_GEMM_EXACT)
        return fail(RR_EINVAL, "unknown engine");
    if (engine == RR_GEMM_EXACT && model != RR_EXACT)
        return fail(RR_EUNSUPPORTED, "the per-sample GEMM engine computes the exact model");
    if (engine == RR_GEMM_EXACT && idx)
        return fail(RR_EUNSUPPORTED, "sampled entries use the direct engine");
    if (engine == RR_GEMM_BF16X3 && model != RR_SEPARABLE)
        return fail(RR_EUNSUPPORTED, "the GEMM engine needs the separable model");
    if (engine == RR_GEMM_BF16X3 && idx)
        return fail(RR_EUNSUPPORTED, "sampled entries use the direct engine");
    const int64_t C = (int64_t)c->ntx * c->nrx, M = c->chirp.n_chirps, K = c->chirp.n_samples;
    const int64_t total = C * M * K;
    if (idx) {
        if (n_idx < 0 || cube_elems < n_idx) return fail(RR_EINVAL, "cube too small for samples");
    } else if (cube_elems < total) {
        return fail(RR_EINVAL, "cube needs %lld complex elements", (long long)total);
    }
    if (C * M > (int64_t)1 << 31) return fail(RR_EUNSUPPORTED, "too many rows");
    HIPCHK(hipSetDevice(c->device));
    const int64_t n = c->n_paths;
    const int shared = c->mode == RR_TX_SHARED;
    const int n_groups = shared ? 1 : c->ntx;
    int rc;
    if ((rc = c->syn.ensure((size_t)std::max<int64_t>(n, 1) * sizeof(SynPath)))) return rc;
    if ((rc = c->ranges.ensure((size_t)(n_groups + 2) * 8))) return rc;
    if (!c->has_scene) return fail(RR_ESTATE, "scene must be set (velocities)");
    if (n > 0) {
        // src must match the launch mode: all -1 (shared) or sorted within [0, n_tx)
        int32_t ends[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(&ends[0], c->paths.soa.src, 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(&ends[1], c->paths.soa.src + (n - 1), 4, hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (shared ? (ends[0] != -1 || ends[1] != -1) : (ends[0] < 0 || ends[1] >= c->ntx))
            return fail(RR_EINVAL, "path sources do not match the array's launch mode");
    }
    SynPath *sp = c->syn.as<SynPath>();
    HIPCHK(launch_syn_prep(c->paths.soa, n, c->obj_vel.as<const double>(), c->nobj,
                           c->pt_vel.as<const double>(), c->npts, sp, c->stream));
    // shared paths carry src = -1: one group over all paths
    if (shared) {
        int64_t r[2] = {0, n};
        HIPCHK(hipMemcpyAsync(c->ranges.p, r, 16, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    } else {
        HIPCHK(launch_ranges(c->paths.soa.src, n, n_groups, 0, c->ranges.as<int64_t>(), c->stream));
    }
    SynthArgs A{};
    A.paths = sp;
    A.ranges = c->ranges.as<const int64_t>();
    A.n_paths = n;
    A.tx = c->tx.as<const double>();
    A.rx = c->rx.as<const double>();
    A.ntx = c->ntx;
    A.nrx = c->nrx;
    for (int a = 0; a < 3; a++) {
        A.oT[a] = c->oT[a];
        A.oR[a] = c->oR[a];
    }
    A.shared = shared;
    A.model = model;
    A.f0 = c->chirp.f0;
    A.bw = c->chirp.bandwidth;
    A.t_rep = c->chirp.t_rep;
    A.inv_c = 1.0 / 299792458.0;
    A.M = (int)M;
    A.K = (int)K;
    A.cube = static_cast<float2 *>(cube);
    if (engine == RR_GEMM_BF16X3) {
        rc = rr_synth_gemm(c, A);
        if (rc) return rc;
    } else if (engine == RR_GEMM_EXACT) {
        rc = rr_synth_freq(c, A);
        if (rc) return rc;
    } else if (idx) {
        HIPCHK(hipEventRecord(c->ev[2], c->stream));
        HIPCHK(launch_synth_sampled(A, idx, n_idx, c->stream));
    } else {
        HIPCHK(hipEventRecord(c->ev[2], c->stream));
        int rows = (int)(shared ? C * M : (int64_t)c->nrx * M);
        hipError_t e = launch_synth_direct(A, n_groups, rows, c->stream);
        if (e == hipErrorInvalidValue) return fail(RR_EUNSUPPORTED, "n_samples too large");
        HIPCHK(e);
    }
    HIPCHK(hipEventRecord(c->ev[3], c->stream));
    c->synth_timed = true;
    g_err.clear();
    return RR_OK;
}

// rr_synthesize with the direct engine over the full cube, allocating
// nothing: the synthesis records and path ranges live in this device's
// scratch; every entry read is written first by this call (no clearing
// needed).  Paths whose source does not belong to the launch mode fall
// outside every range and are not summed.
int rr_synthesize_noalloc(rr_ctx *c, int32_t model, void *cube, int64_t cube_elems)
{
    if (!c || !cube) return fail(RR_EINVAL, "NULL argument");
    if (!c->has_array || !c->has_chirp) return fail(RR_ESTATE, "array and chirp must be set");
    if (!c->has_scene) return fail(RR_ESTATE, "scene must be set (velocities)");
    if (int rc = resolve_paths(c)) return rc;
    if (c->n_paths < 0) return fail(RR_ESTATE, "no paths (trace or rr_set_paths first)");
    if (model != RR_EXACT && model != RR_SEPARABLE) return fail(RR_EINVAL, "unknown model");
    const int64_t C = (int64_t)c->ntx * c->nrx, M = c->chirp.n_chirps, K = c->chirp.n_samples;
    if (cube_elems < C * M * K)
        return fail(RR_EINVAL, "cube needs %lld complex elements", (long long)(C * M * K));
    if (C * M > (int64_t)1 << 31) return fail(RR_EUNSUPPORTED, "too many rows");
    const int64_t n = c->n_paths;
    const int shared = c->mode == RR_TX_SHARED;
    const int n_groups = shared ? 1 : c->ntx;
    if (n > RR_NOALLOC_MAX_PATHS)
        return fail(RR_EUNSUPPORTED, "%lld paths exceed the scratch limit of %d", (long long)n,
                    RR_NOALLOC_MAX_PATHS);
    if (n_groups > RR_NOALLOC_MAX_TX)
        return fail(RR_EUNSUPPORTED, "%d transmitters exceed the scratch limit of %d", n_groups,
                    RR_NOALLOC_MAX_TX);
    HIPCHK(hipSetDevice(c->device));
    unsigned char *base = static_cast<unsigned char *>(g_scratch_dev[c->device]);
    if (!base) return fail(RR_ESTATE, "scratch not initialised on device %d", c->device);
    SynPath *sp = reinterpret_cast<SynPath *>(base);
    int64_t *ranges = reinterpret_cast<int64_t *>(base + NOALLOC_RANGES_OFF);
    HIPCHK(launch_syn_prep(c->paths.soa, n, c->obj_vel.as<const double>(), c->nobj,
                           c->pt_vel.as<const double>(), c->npts, sp, c->stream));
    HIPCHK(launch_ranges(c->paths.soa.src, n, n_groups, shared ? -1 : 0, ranges, c->stream));
    SynthArgs A{};
    A.paths = sp;
    A.ranges = ranges;
    A.n_paths = n;
    A.tx = c->tx.as<const double>();
    A.rx = c->rx.as<const double>();
    A.ntx = c->ntx;
    A.nrx = c->nrx;
    for (int a = 0; a < 3; a++) {
        A.oT[a] = c->oT[a];
        A.oR[a] = c->oR[a];
    }
    A.shared = shared;
    A.model = model;
    A.f0 = c->chirp.f0;
    A.bw = c->chirp.bandwidth;
    A.t_rep = c->chirp.t_rep;
    A.inv_c = 1.0 / 299792458.0;
    A.M = (int)M;
    A.K = (int)K;
    A.cube = static_cast<float2 *>(cube);
    HIPCHK(hipEventRecord(c->ev[2], c->stream));
    const int rows = (int)(shared ? C * M : (int64_t)c->nrx * M);
    hipError_t e = launch_synth_direct(A, n_groups, rows, c->stream);
    if (e == hipErrorInvalidValue) return fail(RR_EUNSUPPORTED, "n_samples too large");
    HIPCHK(e);
    HIPCHK(hipEventRecord(c->ev[3], c->stream));
    c->synth_timed = true;
    g_err.clear();
    return RR_OK;
}

int rr_last_kernel_ms(rr_ctx *c, int32_t which, double *ms)
{
    if (!c || !ms) return fail(RR_EINVAL, "NULL argument");
    if (which < 0 || which > 3 || ((which == 0 || which == 3) && !c->trace_timed) ||
        (which == 1 && !c->synth_timed) || (which == 2 && !c->image_timed))
        return fail(RR_ESTATE, "nothing timed");
    HIPCHK(hipSetDevice(c->device));
    hipEvent_t a = c->ev[which == 3 ? 0 : which * 2], b = c->ev[which == 3 ? 6 : which * 2 + 1];
    HIPCHK(hipEventSynchronize(b));
    float f = 0;
    HIPCHK(hipEventElapsedTime(&f, a, b));
    *ms = f;
    return RR_OK;
}

// --------------------------------------------------------------------------
// imaging
// --------------------------------------------------------------------------

static bool bad_volume(const rr_volume *v)
{
    return !(v->step > 0.0) || !std::isfinite(v->step) || !std::isfinite(v->x0) ||
           !std::isfinite(v->y0) || !std::isfinite(v->z0) || v->nx < 1 || v->ny < 1 || v->nz < 1;
}

int rr_backproject(rr_ctx *c, const void *cube, int64_t cube_elems, const rr_volume *vol,
                   void *image, int64_t image_elems, int32_t engine)
{
    if (!c || !cube || !vol || !image) return fail(RR_EINVAL, "NULL argument");
    if (!c->has_array || !c->has_chirp) return fail(RR_ESTATE, "array and chirp must be set");
    if (bad_volume(vol)) return fail(RR_EINVAL, "invalid voxel grid");
    const int64_t C = (int64_t)c->ntx * c->nrx, M = c->chirp.n_chirps, K = c->chirp.n_samples;
    // the MFMA engine keeps FP32 legs: the phase f d / c must stay below the
    // hardware sin/cos range of 256 turns at the top frequency
    double dmax = 0.0;
    {
        const double cx[2] = {vol->x0, vol->x0 + (vol->nx - 1) * vol->step};
        const double cy[2] = {vol->y0, vol->y0 + (vol->ny - 1) * vol->step};
        const double cz[2] = {vol->z0, vol->z0 + (vol->nz - 1) * vol->step};
        for (int e = 0; e < 2; e++) {
            const std::vector<double> &el = e ? c->h_rx : c->h_tx;
            double m = 0.0;
            for (size_t q = 0; q + 2 < el.size(); q += 3)
                for (int a = 0; a < 8; a++) {
                    const double dx = cx[a & 1] - el[q], dy = cy[(a >> 1) & 1] - el[q + 1],
                                 dz = cz[a >> 2] - el[q + 2];
                    m = std::max(m, std::sqrt(dx * dx + dy * dy + dz * dz));
                }
            dmax = std::max(dmax, m);
        }
    }
    const double fmax = c->chirp.f0 + c->chirp.bandwidth * (double)(K - 1) / (double)K;
    const bool mfma_ok = c->ntx <= 96 && c->nrx <= 96 && dmax * fmax / 299792458.0 < 250.0;
    if (engine == RR_ENGINE_AUTO) engine = mfma_ok ? RR_GEMM_EXACT : RR_DIRECT_FP32;
    if (engine != RR_DIRECT_FP32 && engine != RR_GEMM_EXACT) return fail(RR_EINVAL, "unknown engine");
    if (engine == RR_GEMM_EXACT && !mfma_ok)
        return fail(RR_EUNSUPPORTED, "the MFMA back-projection needs <= 96 Tx and Rx and phases "
                                     "below 250 turns");
    if (engine == RR_DIRECT_FP32 && K > RR_BP_KMAX)
        return fail(RR_EUNSUPPORTED, "sweeps of at most %d steps", RR_BP_KMAX);
    if (cube_elems < C * M * K) return fail(RR_EINVAL, "cube needs %lld complex elements",
                                            (long long)(C * M * K));
    const int64_t nv = (int64_t)vol->nx * vol->ny * vol->nz;
    if (image_elems < nv) return fail(RR_EINVAL, "image needs %lld complex elements", (long long)nv);
    HIPCHK(hipSetDevice(c->device));
    BackProjArgs A{};
    A.cube = static_cast<const float2 *>(cube);
    A.stride = M * K;
    A.tx = c->tx.as<const double>();
    A.rx = c->rx.as<const double>();
    A.ntx = c->ntx;
    A.nrx = c->nrx;
    A.C = (int)C;
    A.K = (int)K;
    A.f0 = c->chirp.f0;
    A.df = c->chirp.bandwidth / (double)K;
    A.inv_c = 1.0 / 299792458.0;
    A.x0 = vol->x0;
    A.y0 = vol->y0;
    A.z0 = vol->z0;
    A.step = vol->step;
    A.nx = vol->nx;
    A.ny = vol->ny;
    A.nz = vol->nz;
    A.n_vox = nv;
    A.image = static_cast<float2 *>(image);
    HIPCHK(hipEventRecord(c->ev[4], c->stream));
    if (engine == RR_GEMM_EXACT) {
        int rc;
        if ((rc = c->bp_sf.ensure((size_t)bp_mfma_frag_bytes((int)K)))) return rc;
        HIPCHK(launch_bp_mfma(A.cube, A.stride, A.tx, c->ntx, A.rx, c->nrx, (int)K, A.f0, A.df,
                              A.inv_c, A.x0, A.y0, A.z0, A.step, A.nx, A.ny, A.nz,
                              c->bp_sf.as<uint4>(), A.image, c->stream));
    } else {
        HIPCHK(launch_backproject(A, c->stream));
    }
    HIPCHK(hipEventRecord(c->ev[5], c->stream));
    c->image_timed = true;
    return RR_OK;
}

int rr_max_projection(rr_ctx *c, const void *image, const rr_volume *vol, float *out,
                      float floor_db)
{
    if (!c || !image || !vol || !out) return fail(RR_EINVAL, "NULL argument");
    if (bad_volume(vol)) return fail(RR_EINVAL, "invalid voxel grid");
    if (!(floor_db <= 0.0f)) return fail(RR_EINVAL, "floor_db must be <= 0");
    HIPCHK(hipSetDevice(c->device));
    int rc;
    if ((rc = c->bp_peak.ensure(256))) return rc;
    HIPCHK(hipMemsetAsync(c->bp_peak.p, 0, 4, c->stream));
    HIPCHK(launch_max_projection(static_cast<const float2 *>(image), vol->nx,
                                 (int64_t)vol->ny * vol->nz, out, c->bp_peak.as<float>(), floor_db,
                                 c->stream));
    return RR_OK;
}

// --------------------------------------------------------------------------
// learned proposal
// --------------------------------------------------------------------------

int rr_proposal_set_cdf(rr_ctx *c, const double *cdf, int32_t n_az, int32_t n_el)
{
    if (!c || !cdf) return fail(RR_EINVAL, "NULL argument");
    if (n_az < 1 || n_el < 1 || (int64_t)n_az * n_el > (1 << 24)) return fail(RR_EINVAL, "bad grid");
    const int64_t nb = (int64_t)n_az * n_el;
    if (cdf[0] != 0.0 || cdf[nb] != 1.0) return fail(RR_EINVAL, "cdf must run from 0 to 1");
    for (int64_t b = 0; b < nb; b++)
        if (!(cdf[b + 1] >= cdf[b])) return fail(RR_EINVAL, "cdf must be non-decreasing");
    HIPCHK(hipSetDevice(c->device));
    int rc = c->cdf.ensure((size_t)(nb + 1) * 8);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(c->cdf.p, cdf, (size_t)(nb + 1) * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->n_az = n_az;
    c->n_el = n_el;
    return RR_OK;
}

int rr_proposal_get_cdf(rr_ctx *c, double *cdf, int64_t cap)
{
    if (!c || !cdf) return fail(RR_EINVAL, "NULL argument");
    if (c->n_az <= 0) return fail(RR_ESTATE, "no proposal table");
    const int64_t n = (int64_t)c->n_az * c->n_el + 1;
    if (cap < n) return fail(RR_EOVERFLOW, "need %lld entries", (long long)n);
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipMemcpyAsync(cdf, c->cdf.p, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return RR_OK;
}

int rr_proposal_probe(rr_ctx *c, double az_min, double az_max, float *code16)
{
    if (!c || !code16) return fail(RR_EINVAL, "NULL argument");
    if (!c->has_scene || !c->has_array) return fail(RR_ESTATE, "scene and array must be set");
    if (!(az_max > az_min) || !std::isfinite(az_min) || !std::isfinite(az_max))
        return fail(RR_EINVAL, "invalid azimuth range");
    HIPCHK(hipSetDevice(c->device));
    TraceArgs A{};
    A.nodes = c->nodes.as<const float4>();
    A.ltris = c->ltris.as<const float4>();
    A.has_bvh = c->n_tris > 0;
    for (int a = 0; a < 3; a++) {
        A.oT[a] = c->oT[a];
        A.oR[a] = c->oR[a];
    }
    const double INV_2PI = 0.15915494309189535;
    A.at = az_min * INV_2PI;
    A.bt = az_max * INV_2PI;
    A.err_flag = c->err_flag.as<int>();
    HIPCHK(launch_probe(A, code16, c->stream));
    return RR_OK;
}

int rr_proposal_histogram(rr_ctx *c, float *hist)
{
    if (!c || !hist) return fail(RR_EINVAL, "NULL argument");
    if (int rc = resolve_paths(c)) return rc;
    if (c->n_paths < 0 || c->last_sampler != RR_UNIFORM || !c->hits_recorded)
        return fail(RR_ESTATE, "needs a uniform trace with record_hits");
    HIPCHK(hipSetDevice(c->device));
    const int nb = RR_PROP_NAZ * RR_PROP_NEL;
    HIPCHK(hipMemsetAsync(hist, 0, (size_t)nb * 4, c->stream));
    HIPCHK(launch_hist(c->last, c->last_traced, c->hits.as<const int32_t>(),
                       c->tri_obj.as<const int32_t>(), RR_PROP_NAZ, RR_PROP_NEL, hist, c->stream));
    return RR_OK;
}

static int mlp_alloc(rr_ctx *c)
{
    int rc;
    if ((rc = c->mlp_p.ensure(RR_MLP_PARAMS * 4))) return rc;
    if ((rc = c->mlp_m.ensure(RR_MLP_PARAMS * 4))) return rc;
    if ((rc = c->mlp_v.ensure(RR_MLP_PARAMS * 4))) return rc;
    if ((rc = c->mlp_g.ensure(RR_MLP_PARAMS * 4))) return rc;
    return RR_OK;
}

static int mlp_reset_adam(rr_ctx *c)
{
    HIPCHK(hipMemsetAsync(c->mlp_m.p, 0, RR_MLP_PARAMS * 4, c->stream));
    HIPCHK(hipMemsetAsync(c->mlp_v.p, 0, RR_MLP_PARAMS * 4, c->stream));
    c->mlp_step = 0;
    return RR_OK;
}

int rr_mlp_set_params(rr_ctx *c, const float *params, int64_t n)
{
    if (!c || !params) return fail(RR_EINVAL, "NULL argument");
    if (n != RR_MLP_PARAMS) return fail(RR_EINVAL, "expected %d parameters", RR_MLP_PARAMS);
    for (int64_t i = 0; i < n; i++)
        if (!std::isfinite(params[i])) return fail(RR_EINVAL, "non-finite parameter");
    HIPCHK(hipSetDevice(c->device));
    int rc = mlp_alloc(c);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(c->mlp_p.p, params, RR_MLP_PARAMS * 4, hipMemcpyHostToDevice, c->stream));
    if ((rc = mlp_reset_adam(c))) return rc;
    HIPCHK(hipStreamSynchronize(c->stream));
    c->mlp_ready = true;
    return RR_OK;
}

int rr_mlp_get_params(rr_ctx *c, float *params, int64_t n)
{
    if (!c || !params) return fail(RR_EINVAL, "NULL argument");
    if (!c->mlp_ready) return fail(RR_ESTATE, "network not initialised");
    if (n < RR_MLP_PARAMS) return fail(RR_EOVERFLOW, "need %d entries", RR_MLP_PARAMS);
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipMemcpyAsync(params, c->mlp_p.p, RR_MLP_PARAMS * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return RR_OK;
}

int rr_mlp_init(rr_ctx *c, uint64_t seed)
{
    if (!c) return fail(RR_EINVAL, "NULL argument");
    // He-uniform: U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)) from a 64-bit LCG
    // (Knuth's MMIX constants), top 53 bits as the uniform
    std::vector<float> p(RR_MLP_PARAMS, 0.0f);
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
    auto uni = [&]() {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(x >> 11) * 0x1.0p-53;
    };
    const int fan[4] = {18, 64, 64, 64}, rows[4] = {64, 64, 64, 1};
    int off = 0;
    for (int l = 0; l < 4; l++) {
        const double lim = std::sqrt(6.0 / fan[l]);
        for (int i = 0; i < rows[l] * fan[l]; i++) p[off + i] = (float)((2.0 * uni() - 1.0) * lim);
        off += rows[l] * fan[l] + rows[l];
    }
    return rr_mlp_set_params(c, p.data(), RR_MLP_PARAMS);
}

static int mlp_buffers(rr_ctx *c, int64_t rows, int n_scenes)
{
    int rc;
    if ((rc = c->mlp_acts.ensure((size_t)rows * 3 * 64 * 2))) return rc;
    if ((rc = c->mlp_z.ensure((size_t)rows * 4))) return rc;
    if ((rc = c->mlp_dz.ensure((size_t)rows * 4))) return rc;
    if ((rc = c->mlp_d.ensure((size_t)rows * 3 * 64 * 4))) return rc;
    if ((rc = c->mlp_loss.ensure((size_t)n_scenes * 4 + 4))) return rc;
    if ((rc = c->mlp_part.ensure((size_t)mlp_part_rows(rows) * RR_MLP_PARAMS * 4))) return rc;
    return RR_OK;
}

int rr_mlp_forward(rr_ctx *c, const float *codes, int32_t n_scenes, float *logits)
{
    if (!c || !codes || !logits) return fail(RR_EINVAL, "NULL argument");
    if (!c->mlp_ready) return fail(RR_ESTATE, "network not initialised");
    if (n_scenes < 1) return fail(RR_EINVAL, "n_scenes must be positive");
    HIPCHK(hipSetDevice(c->device));
    const int64_t rows = (int64_t)n_scenes * RR_PROP_NAZ * RR_PROP_NEL;
    HIPCHK(launch_mlp_forward(c->mlp_p.as<const float>(), codes, rows, nullptr, logits, c->stream));
    return RR_OK;
}

// one Adam step (lr > 0) on n_scenes rows of codes / hist (device); the
// per-scene losses stay in mlp_loss
static int mlp_step(rr_ctx *c, const float *codes, const float *hist, int32_t n_scenes, float lr,
                    float *grad_out)
{
    const int64_t rows = (int64_t)n_scenes * RR_PROP_NAZ * RR_PROP_NEL;
    int rc = mlp_buffers(c, rows, n_scenes);
    if (rc) return rc;
    __half *acts = c->mlp_acts.as<__half>();
    float *d = c->mlp_d.as<float>();
    HIPCHK(launch_mlp_forward(c->mlp_p.as<const float>(), codes, rows, acts, c->mlp_z.as<float>(),
                              c->stream));
    HIPCHK(launch_softmax_grad(c->mlp_z.as<const float>(), hist, n_scenes, c->mlp_dz.as<float>(),
                               c->mlp_loss.as<float>(), c->stream));
    HIPCHK(launch_mlp_backward(c->mlp_p.as<const float>(), c->mlp_dz.as<const float>(), rows, acts,
                               d, d + rows * 64, d + 2 * rows * 64, codes, c->mlp_part.as<float>(),
                               c->mlp_g.as<float>(), c->stream));
    if (grad_out)
        HIPCHK(hipMemcpyAsync(grad_out, c->mlp_g.p, RR_MLP_PARAMS * 4, hipMemcpyDeviceToDevice,
                              c->stream));
    if (lr > 0.0f) {
        c->mlp_step++;
        HIPCHK(launch_adam(c->mlp_p.as<float>(), c->mlp_g.as<const float>(), c->mlp_m.as<float>(),
                           c->mlp_v.as<float>(), lr, c->mlp_step, c->stream));
    }
    return RR_OK;
}

int rr_mlp_train_step(rr_ctx *c, const float *codes, const float *hist, int32_t n_scenes, float lr,
                      float *loss_out, float *grad_out)
{
    if (!c || !codes || !hist) return fail(RR_EINVAL, "NULL argument");
    if (!c->mlp_ready) return fail(RR_ESTATE, "network not initialised");
    if (n_scenes < 1) return fail(RR_EINVAL, "n_scenes must be positive");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(RR_EINVAL, "invalid learning rate");
    HIPCHK(hipSetDevice(c->device));
    int rc = mlp_step(c, codes, hist, n_scenes, lr, grad_out);
    if (rc) return rc;
    if (loss_out) {
        std::vector<float> l(n_scenes);
        HIPCHK(hipMemcpyAsync(l.data(), c->mlp_loss.p, (size_t)n_scenes * 4, hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        double s = 0.0;
        for (float v : l) s += v;
        *loss_out = (float)s;
    }
    return RR_OK;
}

// SplitMix64 (Steele, Lea and Flood 2014)
static uint64_t splitmix64(uint64_t &x)
{
    uint64_t z = (x += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

int rr_proposal_train(rr_ctx *c, const float *codes, const float *hist, int32_t n_scenes,
                      int32_t steps, int32_t batch, float lr, uint64_t seed, float *loss_out)
{
    if (!c || !codes || !hist) return fail(RR_EINVAL, "NULL argument");
    if (!c->mlp_ready) return fail(RR_ESTATE, "network not initialised");
    if (n_scenes < 1 || steps < 0 || batch < 1)
        return fail(RR_EINVAL, "n_scenes and batch must be positive, steps non-negative");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(RR_EINVAL, "invalid learning rate");
    HIPCHK(hipSetDevice(c->device));
    const int B = std::min(batch, n_scenes);
    const int64_t nb = RR_PROP_NAZ * RR_PROP_NEL;
    int rc;
    if ((rc = mlp_buffers(c, (int64_t)B * nb, B))) return rc;
    const bool gather = B < n_scenes;
    if (gather) {
        if ((rc = c->tr_codes.ensure((size_t)B * 16 * 4))) return rc;
        if ((rc = c->tr_hist.ensure((size_t)B * nb * 4))) return rc;
    }
    if (loss_out && steps > 0 && (rc = c->tr_loss.ensure((size_t)steps * B * 4))) return rc;
    std::vector<int32_t> perm(n_scenes);
    for (int32_t i = 0; i < n_scenes; i++) perm[i] = i;
    uint64_t st = seed;
    for (int32_t s = 0; s < steps; s++) {
        const float *cb = codes, *hb = hist;
        if (gather) {
            // B distinct scenes: the first B entries of a partial Fisher-Yates shuffle
            for (int k = 0; k < B; k++) {
                const int j = k + (int)(splitmix64(st) % (uint64_t)(n_scenes - k));
                std::swap(perm[k], perm[j]);
                HIPCHK(hipMemcpyAsync(c->tr_codes.as<float>() + (int64_t)k * 16,
                                      codes + (int64_t)perm[k] * 16, 16 * 4,
                                      hipMemcpyDeviceToDevice, c->stream));
                HIPCHK(hipMemcpyAsync(c->tr_hist.as<float>() + (int64_t)k * nb,
                                      hist + (int64_t)perm[k] * nb, (size_t)nb * 4,
                                      hipMemcpyDeviceToDevice, c->stream));
            }
            cb = c->tr_codes.as<const float>();
            hb = c->tr_hist.as<const float>();
        }
        if ((rc = mlp_step(c, cb, hb, B, lr, nullptr))) return rc;
        if (loss_out)
            HIPCHK(hipMemcpyAsync(c->tr_loss.as<float>() + (int64_t)s * B, c->mlp_loss.p,
                                  (size_t)B * 4, hipMemcpyDeviceToDevice, c->stream));
    }
    if (loss_out && steps > 0) {
        std::vector<float> l((size_t)steps * B);
        HIPCHK(hipMemcpyAsync(l.data(), c->tr_loss.p, l.size() * 4, hipMemcpyDeviceToHost,
                              c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int32_t s = 0; s < steps; s++) {
            double sum = 0.0;
            for (int k = 0; k < B; k++) sum += l[(size_t)s * B + k];
            loss_out[s] = (float)sum;
        }
    }
    return RR_OK;
}

static int proposal_table(rr_ctx *c, const float *code16, float beta, float power, float kappa)
{
    HIPCHK(hipSetDevice(c->device));
    const int nb = RR_PROP_NAZ * RR_PROP_NEL;
    int rc;
    if ((rc = c->mlp_z.ensure((size_t)nb * 4))) return rc;
    if ((rc = c->cdf.ensure((size_t)(nb + 1) * 8))) return rc;
    HIPCHK(launch_mlp_forward(c->mlp_p.as<const float>(), code16, nb, nullptr, c->mlp_z.as<float>(),
                              c->stream));
    HIPCHK(launch_build_cdf(c->mlp_z.as<const float>(), beta, power, kappa, c->cdf.as<double>(),
                            c->stream));
    c->n_az = RR_PROP_NAZ;
    c->n_el = RR_PROP_NEL;
    return RR_OK;
}

int rr_proposal_build(rr_ctx *c, const float *code16, float beta, float power)
{
    if (!c || !code16) return fail(RR_EINVAL, "NULL argument");
    if (!c->mlp_ready) return fail(RR_ESTATE, "network not initialised");
    if (!(beta >= 0.0f && beta <= 1.0f)) return fail(RR_EINVAL, "beta must be in [0, 1]");
    if (!(power > 0.0f && power <= 2.0f)) return fail(RR_EINVAL, "power must be in (0, 2]");
    return proposal_table(c, code16, beta, power, 0.0f);
}

int rr_proposal_build_cost(rr_ctx *c, const float *code16, float beta, float kappa)
{
    if (!c || !code16) return fail(RR_EINVAL, "NULL argument");
    if (!c->mlp_ready) return fail(RR_ESTATE, "network not initialised");
    if (!(beta >= 0.0f && beta <= 1.0f)) return fail(RR_EINVAL, "beta must be in [0, 1]");
    if (!(kappa > 0.0f) || !std::isfinite(kappa)) return fail(RR_EINVAL, "kappa must be positive");
    return proposal_table(c, code16, beta, 1.0f, kappa);
}

// --------------------------------------------------------------------------
// batched launch
// --------------------------------------------------------------------------

}  // extern "C"

namespace {

struct BatchScene {
    bool set = false;
    int64_t n_tris = 0;
    int nobj = 0, npts = 0, ntx = 0, nrx = 0, mode = 0;
    double rx_radius = 0.25, oT[3] = {0, 0, 0}, oR[3] = {0, 0, 0};
    DevBuf nodes, ltris, obj_alpha, obj_vel, pt_pos, pt_vel, pt_ap, tx, rx;
    rr_chirp chirp{};
    rr_trace_params tp{};
    int64_t n_src = 0, n_per_src = 0, n_vps = 0, V = 0;
    int kr = 0;
    // synthesis engine: requested (RR_ENGINE_AUTO, RR_DIRECT_FP32 or
    // RR_GEMM_EXACT, product tile 0 or 16/32/48/64/96), the autotuner's
    // choice for AUTO (-1: not tuned), and the plan of the current graph
    int req_engine = RR_ENGINE_AUTO, req_tile = 0;
    int tuned_engine = -1, tuned_tile = 0;
    int try_engine = -1, try_tile = 0;    // forced plan while the tuner times a candidate
    bool use_freq = false;
    int tile = 0;                         // exact engine: product tile
    int64_t fq_cap = 0;                   // exact engine: leg table capacity (paths)
    int fq_split = 1;
    int64_t fq_ppad = 0, fq_split_len = 0;  // table stride and split length of the graph
    int64_t n_last = -1;                  // path count of the last launch
    void release()
    {
        DevBuf *b[] = {&nodes, &ltris, &obj_alpha, &obj_vel, &pt_pos, &pt_vel, &pt_ap, &tx, &rx};
        for (DevBuf *x : b) x->release();
    }
};

int largest_kr(int K, int limit)
{
    int kr = limit;
    while (kr > 1 && (K % kr != 0 || K / kr > 256)) kr >>= 1;
    return (K / kr > 256) ? 0 : kr;
}

}  // namespace

struct rr_batch {
    rr_ctx *c = nullptr;
    int S = 0;
    std::vector<BatchScene> sc;
    hipStream_t st = nullptr;
    hipEvent_t ev[6] = {};
    DevBuf d_targs, d_sargs, d_info, d_chunk, d_items, d_vr, d_vel, d_rinfo, d_ranges;
    DevBuf counts, offsets, bsums, total, counter, work;
    PathStore tmp, fin;
    DevBuf syn, alpha_tmp;
    DevBuf fq_xt, fq_yt, fq_amp, fq_src, fq_part;   // exact engine, shared by its scenes
    int64_t cap = 0, V_total = 0, n_chunks = 0, n_items = 0, n_ranges = 0, nb = 0;
    std::vector<char> synth_on;           // scenes the synthesis stage computes
    std::vector<int64_t> range_base;
    std::vector<void *> cubes;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool dirty = true;
    float ms_trace = 0, ms_synth = 0, ms_total = 0;   // stages: last eager run; total: last launch
    int64_t last_total = 0;
};

namespace {

void batch_drop_graph(rr_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->dirty = true;
}

// leg table bytes of the exact engine for a scene at a path capacity and
// product layout
int64_t batch_freq_bytes(const BatchScene &x, int64_t cap, int tile)
{
    const bool own = freq_own_tx(tile, x.mode != RR_TX_SHARED, true);
    return 8 * freq_table_entries(x.ntx, x.nrx, x.chirp.n_chirps, cap, own);
}

// the exact engine's table budget for AUTO in a batch (the tables are shared
// by the scenes that use it, one after the other)
const int64_t BATCH_FREQ_TABLE_MAX = (int64_t)16 << 30;

// the synthesis plan of scene x: the exact product engine (and its tile) or
// the direct engine, and the exact engine's table capacity
void batch_plan(BatchScene &x)
{
    const int64_t ks = freq_k_step();
    const int64_t est = x.n_src * x.n_per_src / 16 + x.n_src * x.npts;
    const int64_t want = x.n_last >= 0 ? x.n_last + x.n_last / 4 + 1024 : est;
    // start from the estimate; follow the last launch's count down when the
    // capacity is more than twice what it needs (growth comes from overflow)
    if (x.fq_cap <= 0 || x.fq_cap > 2 * want) x.fq_cap = want;
    x.fq_cap = std::max<int64_t>((x.fq_cap + ks - 1) / ks * ks, ks);
    int eng = x.req_engine, tile = x.req_tile;
    if (x.try_engine >= 0) {
        eng = x.try_engine;
        tile = x.try_tile;
    } else if (eng == RR_ENGINE_AUTO && x.tuned_engine >= 0) {
        eng = x.tuned_engine;
        tile = x.tuned_tile;
    }
    const int K = x.chirp.n_samples;
    const bool per_el = x.mode != RR_TX_SHARED;
    if (tile <= 0) tile = freq_tile(x.ntx, x.nrx, K, per_el);
    if (eng == RR_ENGINE_AUTO) {
        // untuned: the single-scene rule (the product layout pays), within
        // the table budget
        eng = freq_pays(x.ntx, x.nrx, K, per_el) && batch_freq_bytes(x, x.fq_cap, tile) <= BATCH_FREQ_TABLE_MAX
                  ? RR_GEMM_EXACT
                  : RR_DIRECT_FP32;
    }
    if (tile == 1 && K > 1024) tile = freq_tile(x.ntx, x.nrx, K, per_el);   // no sample split that long
    x.use_freq = eng == RR_GEMM_EXACT;
    x.tile = tile;
}

// per-scene tables and global buffers for the current scene set and cubes;
// only_K > 0 gives synthesis work to the scenes with that sample count alone,
// only_scene >= 0 to that scene alone, and p_limit > 0 caps the paths of each
// group (all three for the autotuner's timing)
int batch_prepare(rr_batch *b, int only_K = 0, int64_t p_limit = 0, int only_scene = -1)
{
    const int S = b->S;
    std::vector<TraceArgs> ta(S);
    std::vector<SynthArgs> sa(S);
    std::vector<BatchSynthInfo> info(S);
    std::vector<BatchVel> vel(S);
    std::vector<BatchRangeInfo> ri(S);
    std::vector<int64_t> chunk(S + 1, 0), items(S + 1, 0), vr(S + 1, 0);
    b->range_base.assign(S + 1, 0);
    b->synth_on.assign(S, 0);
    int64_t V = 0, est = 0;
    for (int s = 0; s < S; s++) {
        BatchScene &x = b->sc[s];
        if (!x.set) return fail(RR_ESTATE, "batch slot %d is empty", s);
        const int shared = x.mode == RR_TX_SHARED;
        x.n_src = shared ? 1 : x.ntx;
        x.n_per_src = shared ? x.tp.n_rays : x.tp.n_rays / x.ntx;
        x.n_vps = x.n_per_src + x.npts;
        x.V = x.n_src * x.n_vps;
        vr[s] = V;
        V += x.V;
        est += x.n_src * x.n_per_src / 16 + x.n_src * x.npts;
        const int64_t rchunks = (x.n_src * x.n_per_src + RR_TRACE_BLOCK - 1) / RR_TRACE_BLOCK;
        const int64_t pchunks = (x.n_src * x.npts + RR_TRACE_BLOCK - 1) / RR_TRACE_BLOCK;
        chunk[s + 1] = chunk[s] + rchunks + pchunks;
        const int K = x.chirp.n_samples, M = x.chirp.n_chirps;
        if (x.kr <= 0) x.kr = largest_kr(K, RR_BATCH_MAX_KR);
        if (x.kr <= 0) return fail(RR_EUNSUPPORTED, "scene %d: n_samples too large", s);
        const int n_groups = shared ? 1 : x.ntx;
        const int RC = shared ? x.ntx * x.nrx : x.nrx;
        const int rows = RC * M;
        const int RPB = 256 / (K / x.kr);
        info[s].kr = x.kr;
        info[s].rows_per_group = rows;
        info[s].rc = RC;
        info[s].bpg = (rows + RPB - 1) / RPB;
        batch_plan(x);
        const bool synth = (only_K <= 0 || K == only_K) && (only_scene < 0 || s == only_scene);
        b->synth_on[s] = synth;
        items[s + 1] = items[s] + (synth && !x.use_freq ? (int64_t)info[s].bpg * n_groups : 0);
        b->range_base[s + 1] = b->range_base[s] + (shared ? 2 : n_groups + 1);
    }
    vr[S] = V;
    if (V >= (int64_t(1) << 32)) return fail(RR_EUNSUPPORTED, "too many rays in the batch");
    if (b->cap == 0) b->cap = std::max<int64_t>(65536, est);
    b->V_total = V;
    b->n_chunks = chunk[S];
    b->n_items = items[S];
    b->n_ranges = b->range_base[S];
    b->nb = scan_u8_blocks(V);
    int rc;
    if ((rc = b->counts.ensure((size_t)V + 64))) return rc;
    if ((rc = b->offsets.ensure((size_t)V * 4 + 64))) return rc;
    if ((rc = b->bsums.ensure((size_t)(b->nb + 1) * 4))) return rc;
    if ((rc = b->total.ensure(256))) return rc;
    if ((rc = b->counter.ensure(256))) return rc;
    if ((rc = b->work.ensure(256))) return rc;
    if ((rc = b->tmp.alloc(b->cap))) return rc;
    if ((rc = b->fin.alloc(b->cap))) return rc;
    if ((rc = b->syn.ensure((size_t)b->cap * sizeof(SynPath)))) return rc;
    if ((rc = b->d_targs.ensure(sizeof(TraceArgs) * S))) return rc;
    if ((rc = b->d_sargs.ensure(sizeof(SynthArgs) * S))) return rc;
    if ((rc = b->d_info.ensure(sizeof(BatchSynthInfo) * S))) return rc;
    if ((rc = b->d_vel.ensure(sizeof(BatchVel) * S))) return rc;
    if ((rc = b->d_rinfo.ensure(sizeof(BatchRangeInfo) * S))) return rc;
    if ((rc = b->d_chunk.ensure(8 * (S + 1)))) return rc;
    if ((rc = b->d_items.ensure(8 * (S + 1)))) return rc;
    if ((rc = b->d_vr.ensure(8 * (S + 1)))) return rc;
    if ((rc = b->d_ranges.ensure(8 * (b->n_ranges + 1)))) return rc;
    // exact engine: per scene the table stride (capacity, or the timing cap)
    // and path splits; one set of tables serves its scenes in turn
    {
        const int64_t ks = freq_k_step();
        size_t xt = 0, yt = 0, pp = 0, part = 0;
        for (int s = 0; s < S; s++) {
            BatchScene &x = b->sc[s];
            if (!x.use_freq || !b->synth_on[s]) continue;
            int64_t P = x.fq_cap;
            if (p_limit > 0) P = std::min<int64_t>(P, std::max<int64_t>((p_limit + ks - 1) / ks * ks, ks));
            x.fq_ppad = P;
            const int M = x.chirp.n_chirps, K = x.chirp.n_samples;
            freq_splits(x.tile, x.ntx, x.nrx, M, K, P, x.fq_split, x.fq_split_len);
            const bool own = freq_own_tx(x.tile, x.mode != RR_TX_SHARED, true);
            xt = std::max(xt, (size_t)M * (own ? 1 : x.ntx) * P * 8);
            yt = std::max(yt, (size_t)M * x.nrx * P * 8);
            pp = std::max(pp, (size_t)P * 4);
            if (x.fq_split > 1)
                part = std::max(part, (size_t)x.fq_split * M * K * x.ntx * x.nrx * 8);
        }
        if (pp) {
            if ((rc = b->fq_xt.ensure(xt))) return rc;
            if ((rc = b->fq_yt.ensure(yt))) return rc;
            if ((rc = b->fq_amp.ensure(pp))) return rc;
            if ((rc = b->fq_src.ensure(pp))) return rc;
            if (part && (rc = b->fq_part.ensure(part))) return rc;
        }
    }
    const double INV_2PI = 0.15915494309189535;
    for (int s = 0; s < S; s++) {
        BatchScene &x = b->sc[s];
        TraceArgs &A = ta[s];
        A = TraceArgs{};
        A.nodes = x.nodes.as<const float4>();
        A.ltris = x.ltris.as<const float4>();
        A.has_bvh = x.n_tris > 0;
        A.tx = x.tx.as<const double>();
        A.pt_pos = x.pt_pos.as<const double>();
        A.pt_ap = x.pt_ap.as<const double>();
        for (int a = 0; a < 3; a++) {
            A.oT[a] = x.oT[a];
            A.oR[a] = x.oR[a];
        }
        A.r2 = x.rx_radius * x.rx_radius;
        A.shared = x.mode == RR_TX_SHARED;
        A.nobj = x.nobj;
        A.npts = x.npts;
        A.n_src = x.n_src;
        A.n_per_src = x.n_per_src;
        A.n_virt_per_src = x.n_vps;
        A.at = x.tp.az_min * INV_2PI;
        A.bt = x.tp.az_max * INV_2PI;
        A.slo = std::sin(x.tp.el_min);
        A.shi = std::sin(x.tp.el_max);
        A.omega = (x.tp.az_max - x.tp.az_min) * (A.shi - A.slo);
        A.bmax = x.tp.max_bounces;
        A.seed = x.tp.seed;
        A.sampler = RR_UNIFORM;
        A.vbase = vr[s];
        A.hits = nullptr;
        A.counts = b->counts.as<uint8_t>();
        A.tmp = b->tmp.soa;
        A.counter = b->counter.as<unsigned long long>();
        A.err_flag = b->c->err_flag.as<int>();
        SynthArgs &Y = sa[s];
        Y = SynthArgs{};
        Y.paths = b->syn.as<const SynPath>();
        Y.ranges = b->d_ranges.as<const int64_t>() + b->range_base[s];
        Y.n_paths = 0;
        Y.tx = x.tx.as<const double>();
        Y.rx = x.rx.as<const double>();
        Y.ntx = x.ntx;
        Y.nrx = x.nrx;
        for (int a = 0; a < 3; a++) {
            Y.oT[a] = x.oT[a];
            Y.oR[a] = x.oR[a];
        }
        Y.shared = x.mode == RR_TX_SHARED;
        Y.model = RR_EXACT;
        Y.f0 = x.chirp.f0;
        Y.bw = x.chirp.bandwidth;
        Y.t_rep = x.chirp.t_rep;
        Y.inv_c = 1.0 / 299792458.0;
        Y.M = x.chirp.n_chirps;
        Y.K = x.chirp.n_samples;
        Y.cube = static_cast<float2 *>(s < (int)b->cubes.size() ? b->cubes[s] : nullptr);
        Y.p_limit = p_limit;
        vel[s].obj_vel = x.obj_vel.as<const double>();
        vel[s].pt_vel = x.pt_vel.as<const double>();
        vel[s].nobj = x.nobj;
        vel[s].npts = x.npts;
        ri[s].vr0 = vr[s];
        ri[s].n_vps = x.n_vps;
        ri[s].base = b->range_base[s];
        ri[s].n_groups = (int)x.n_src;
        ri[s].shared = x.mode == RR_TX_SHARED;
    }
    hipStream_t st = b->st;
    HIPCHK(hipMemcpyAsync(b->d_targs.p, ta.data(), sizeof(TraceArgs) * S, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->d_sargs.p, sa.data(), sizeof(SynthArgs) * S, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->d_info.p, info.data(), sizeof(BatchSynthInfo) * S, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->d_vel.p, vel.data(), sizeof(BatchVel) * S, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->d_rinfo.p, ri.data(), sizeof(BatchRangeInfo) * S, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->d_chunk.p, chunk.data(), 8 * (S + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->d_items.p, items.data(), 8 * (S + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(b->d_vr.p, vr.data(), 8 * (S + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return RR_OK;
}

// the trace stage: zero the queue and path counters (kernel fills, no
// memset nodes), persistent trace, scan, scatter, synthesis records, ranges
int batch_enqueue_trace(rr_batch *b, bool timed)
{
    hipStream_t st = b->st;
    unsigned long long *work = b->work.as<unsigned long long>();
    HIPCHK(launch_fill_u64(work, 2, 0ull, st));
    HIPCHK(launch_fill_u64(b->counter.as<unsigned long long>(), 1, 0ull, st));
    if (timed) HIPCHK(hipEventRecord(b->ev[0], st));
    HIPCHK(launch_batch_trace(b->d_targs.as<const TraceArgs>(), b->d_chunk.as<const int64_t>(), b->S,
                              b->n_chunks, work, st));
    HIPCHK(launch_scan_u8(b->counts.as<const uint8_t>(), b->V_total, b->offsets.as<uint32_t>(),
                          b->bsums.as<uint32_t>(), b->nb + 1, b->total.as<unsigned long long>(), st));
    HIPCHK(launch_scatter(b->tmp.soa, b->counter.as<const unsigned long long>(), b->cap,
                          b->offsets.as<const uint32_t>(), b->fin.soa, b->cap, st));
    HIPCHK(launch_batch_prep(b->fin.soa, b->total.as<const unsigned long long>(), b->cap,
                             b->d_vr.as<const int64_t>(), b->S, b->d_vel.as<const BatchVel>(),
                             b->syn.as<SynPath>(), st));
    HIPCHK(launch_batch_ranges(b->offsets.as<const uint32_t>(), b->V_total,
                               b->total.as<const unsigned long long>(), b->cap,
                               b->d_rinfo.as<const BatchRangeInfo>(), b->S, b->d_ranges.as<int64_t>(),
                               st));
    if (timed) HIPCHK(hipEventRecord(b->ev[1], st));
    return RR_OK;
}

int batch_enqueue_synth(rr_batch *b, bool timed)
{
    hipStream_t st = b->st;
    unsigned long long *work = b->work.as<unsigned long long>();
    HIPCHK(launch_fill_u64(work + 1, 1, 0ull, st));
    if (timed) HIPCHK(hipEventRecord(b->ev[2], st));
    HIPCHK(launch_batch_synth(b->d_sargs.as<const SynthArgs>(), b->d_info.as<const BatchSynthInfo>(),
                              b->d_items.as<const int64_t>(), b->S, b->n_items, work + 1, st));
    // the exact product engine's scenes, one after the other on the shared
    // tables; each reads its path range from the device
    const int64_t *rg = b->d_ranges.as<const int64_t>();
    for (int s = 0; s < b->S; s++) {
        const BatchScene &x = b->sc[s];
        if (!x.use_freq || !b->synth_on[s]) continue;
        const int64_t *lo = rg + b->range_base[s], *hi = rg + b->range_base[s + 1] - 1;
        const int M = x.chirp.n_chirps, K = x.chirp.n_samples;
        const double inv_c = 1.0 / 299792458.0;
        HIPCHK(launch_freq_prep(b->syn.as<const SynPath>(), 0, lo, hi, x.fq_ppad, M, x.chirp.t_rep,
                                x.tx.as<const double>(), x.ntx,
                                freq_own_tx(x.tile, x.mode != RR_TX_SHARED, true),
                                x.rx.as<const double>(), x.nrx, x.chirp.f0 * inv_c,
                                x.chirp.bandwidth / (double)K * inv_c, b->fq_xt.as<uint2>(),
                                b->fq_yt.as<uint2>(),
                                b->fq_amp.as<float>(), b->fq_src.as<int32_t>(), st));
        HIPCHK(launch_freq_gemm(b->fq_xt.as<const uint2>(), b->fq_yt.as<const uint2>(),
                                b->fq_amp.as<const float>(), b->fq_src.as<const int32_t>(), x.ntx,
                                x.nrx, M, K, x.fq_ppad, x.fq_split, x.fq_split_len,
                                x.mode != RR_TX_SHARED, x.tile, lo, hi, lo, b->fq_part.as<float2>(),
                                static_cast<float2 *>(b->cubes[s]), st));
    }
    if (timed) HIPCHK(hipEventRecord(b->ev[3], st));
    return RR_OK;
}

// after a launch: the path pool and every exact-engine scene's table
// capacity against the counts; a shortfall grows the capacity and asks for a
// re-run (*overflow).  Records each scene's path count.
int batch_check(rr_batch *b, bool *overflow)
{
    unsigned long long cnt = 0, tot = 0;
    std::vector<int64_t> r(b->n_ranges + 1);
    HIPCHK(hipMemcpyAsync(&cnt, b->counter.p, 8, hipMemcpyDeviceToHost, b->st));
    HIPCHK(hipMemcpyAsync(&tot, b->total.p, 8, hipMemcpyDeviceToHost, b->st));
    HIPCHK(hipMemcpyAsync(r.data(), b->d_ranges.p, 8 * b->n_ranges, hipMemcpyDeviceToHost, b->st));
    HIPCHK(hipStreamSynchronize(b->st));
    *overflow = (int64_t)cnt > b->cap;
    if (*overflow) b->cap = (int64_t)cnt + (int64_t)cnt / 4 + 4096;
    b->last_total = (int64_t)tot;
    if (*overflow) return RR_OK;   // counts are cut short: re-run first
    for (int s = 0; s < b->S; s++) {
        BatchScene &x = b->sc[s];
        const int64_t n = r[b->range_base[s + 1] - 1] - r[b->range_base[s]];
        x.n_last = n;
        if (x.use_freq && b->synth_on[s] && n > x.fq_ppad) {
            x.fq_cap = n + n / 4 + 1024;
            *overflow = true;
        }
    }
    return RR_OK;
}

bool batch_any_freq(const rr_batch *b)
{
    for (const auto &x : b->sc)
        if (x.use_freq) return true;
    return false;
}

}  // namespace

extern "C" {

int rr_batch_create(rr_ctx *c, int32_t n_scenes, rr_batch **out)
{
    if (!c || !out) return fail(RR_EINVAL, "NULL argument");
    if (n_scenes < 1) return fail(RR_EINVAL, "n_scenes must be positive");
    HIPCHK(hipSetDevice(c->device));
    rr_batch *b = new rr_batch();
    b->c = c;
    b->S = n_scenes;
    b->sc.resize(n_scenes);
    if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return fail(RR_EHIP, "hipStreamCreate failed");
    }
    for (auto &e : b->ev) HIPCHK(hipEventCreate(&e));
    *out = b;
    return RR_OK;
}

void rr_batch_destroy(rr_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->c->device);
    if (b->st) (void)hipStreamSynchronize(b->st);
    batch_drop_graph(b);
    for (auto &x : b->sc) x.release();
    DevBuf *bufs[] = {&b->d_targs, &b->d_sargs, &b->d_info, &b->d_chunk, &b->d_items, &b->d_vr,
                      &b->d_vel, &b->d_rinfo, &b->d_ranges, &b->counts, &b->offsets, &b->bsums,
                      &b->total, &b->counter, &b->work, &b->syn, &b->alpha_tmp, &b->tmp.buf,
                      &b->fin.buf};
    for (DevBuf *x : bufs) x->release();
    for (auto &e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->st) (void)hipStreamDestroy(b->st);
    delete b;
}

int rr_batch_set_scene(rr_batch *b, int32_t slot, const float *verts, int64_t n_verts,
                       const int32_t *tris, const int32_t *tri_obj, int64_t n_tris,
                       const float *obj_alpha, const double *obj_vel, int32_t n_obj,
                       const double *pt_pos, const double *pt_vel, const double *pt_aperture,
                       int32_t n_pts, const double *tx, int32_t n_tx, const double *rx, int32_t n_rx,
                       double rx_radius, int32_t tx_mode, const rr_chirp *chirp,
                       const rr_trace_params *tp)
{
    if (!b || !chirp || !tp) return fail(RR_EINVAL, "NULL argument");
    if (slot < 0 || slot >= b->S) return fail(RR_EINVAL, "slot out of range");
    // validate through the single-scene entry points on a scratch check
    if (n_verts < 0 || n_tris < 0 || n_obj < 1 || n_pts < 0)
        return fail(RR_EINVAL, "negative size or no object");
    if ((n_tris > 0 && (!verts || !tris || !tri_obj)) || !obj_alpha || !obj_vel ||
        (n_pts > 0 && (!pt_pos || !pt_vel || !pt_aperture)) || !tx || !rx || n_tx < 1 || n_rx < 1)
        return fail(RR_EINVAL, "NULL array");
    for (int64_t i = 0; i < 3 * n_verts; i++)
        if (!std::isfinite(verts[i])) return fail(RR_EINVAL, "non-finite vertex coordinate");
    for (int64_t i = 0; i < n_tris; i++) {
        for (int k = 0; k < 3; k++)
            if (tris[3 * i + k] < 0 || tris[3 * i + k] >= n_verts)
                return fail(RR_EINVAL, "triangle vertex index out of range");
        if (tri_obj[i] < 0 || tri_obj[i] >= n_obj) return fail(RR_EINVAL, "triangle object out of range");
    }
    for (int i = 0; i < n_obj; i++)
        if (!(obj_alpha[i] >= 0.0f && obj_alpha[i] <= 1.0f)) return fail(RR_EINVAL, "alpha outside [0, 1]");
    if (!finite3(obj_vel, n_obj) || (n_pts > 0 && (!finite3(pt_pos, n_pts) || !finite3(pt_vel, n_pts))) ||
        !finite3(tx, n_tx) || !finite3(rx, n_rx))
        return fail(RR_EINVAL, "non-finite input");
    if (!(rx_radius > 0.0) || (tx_mode != RR_TX_PER_ELEMENT && tx_mode != RR_TX_SHARED))
        return fail(RR_EINVAL, "invalid array");
    if (!(chirp->f0 > 0.0) || !(chirp->bandwidth >= 0.0) || !(chirp->t_chirp > 0.0) ||
        !(chirp->t_rep >= 0.0) || chirp->n_samples < 1 || chirp->n_chirps < 1)
        return fail(RR_EINVAL, "degenerate chirp");
    if (tp->max_bounces < 1 || tp->max_bounces > RR_KMAX || tp->n_rays < 0 ||
        !(tp->az_max > tp->az_min) || !(tp->el_max > tp->el_min) || tp->sampler != RR_UNIFORM)
        return fail(RR_EINVAL, "invalid trace parameters (batched traces use the uniform sampler)");
    if (largest_kr(chirp->n_samples, 32) <= 0) return fail(RR_EUNSUPPORTED, "n_samples too large");
    HIPCHK(hipSetDevice(b->c->device));
    HIPCHK(hipStreamSynchronize(b->st));
    HostBvh bvh;
    std::string err;
    int rc = rr_build_bvh(verts, n_verts, tris, tri_obj, obj_alpha, n_tris, bvh, err);
    if (rc) return fail(rc, "BVH build: %s", err.c_str());
    BatchScene &x = b->sc[slot];
    if ((rc = x.nodes.ensure(bvh.nodes.size() * 4 + 64))) return rc;
    if ((rc = x.ltris.ensure(bvh.tris.size() * 4 + 64))) return rc;
    if ((rc = x.obj_alpha.ensure((size_t)n_obj * 4))) return rc;
    if ((rc = x.obj_vel.ensure((size_t)n_obj * 24))) return rc;
    if ((rc = x.pt_pos.ensure((size_t)n_pts * 24 + 8))) return rc;
    if ((rc = x.pt_vel.ensure((size_t)n_pts * 24 + 8))) return rc;
    if ((rc = x.pt_ap.ensure((size_t)n_pts * 8 + 8))) return rc;
    if ((rc = x.tx.ensure((size_t)n_tx * 24))) return rc;
    if ((rc = x.rx.ensure((size_t)n_rx * 24))) return rc;
    if (!bvh.nodes.empty()) HIPCHK(hipMemcpy(x.nodes.p, bvh.nodes.data(), bvh.nodes.size() * 4, hipMemcpyHostToDevice));
    if (!bvh.tris.empty()) HIPCHK(hipMemcpy(x.ltris.p, bvh.tris.data(), bvh.tris.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(x.obj_alpha.p, obj_alpha, (size_t)n_obj * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(x.obj_vel.p, obj_vel, (size_t)n_obj * 24, hipMemcpyHostToDevice));
    if (n_pts > 0) {
        HIPCHK(hipMemcpy(x.pt_pos.p, pt_pos, (size_t)n_pts * 24, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(x.pt_vel.p, pt_vel, (size_t)n_pts * 24, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(x.pt_ap.p, pt_aperture, (size_t)n_pts * 8, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(x.tx.p, tx, (size_t)n_tx * 24, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(x.rx.p, rx, (size_t)n_rx * 24, hipMemcpyHostToDevice));
    for (int a = 0; a < 3; a++) {
        double st = 0.0, sr = 0.0;
        for (int i = 0; i < n_tx; i++) st += tx[3 * i + a];
        for (int i = 0; i < n_rx; i++) sr += rx[3 * i + a];
        x.oT[a] = st / (double)n_tx;
        x.oR[a] = sr / (double)n_rx;
    }
    x.n_tris = n_tris;
    x.nobj = n_obj;
    x.npts = n_pts;
    x.ntx = n_tx;
    x.nrx = n_rx;
    x.mode = tx_mode;
    x.rx_radius = rx_radius;
    x.chirp = *chirp;
    x.tp = *tp;
    x.kr = 0;
    x.tuned_engine = -1;
    x.n_last = -1;
    x.fq_cap = 0;
    x.set = true;
    batch_drop_graph(b);
    return RR_OK;
}

int rr_batch_set_alpha(rr_batch *b, int32_t slot, const float *alpha, int64_t n, int32_t per)
{
    if (!b) return fail(RR_EINVAL, "NULL batch");
    if (slot < 0 || slot >= b->S) return fail(RR_EINVAL, "slot out of range");
    BatchScene &x = b->sc[slot];
    if (!x.set) return fail(RR_ESTATE, "slot %d has no scene", slot);
    HIPCHK(hipSetDevice(b->c->device));
    // the captured launch reads the leaf records in place: no re-capture needed
    int rc = set_alpha_common(b->st, x.ltris, x.obj_alpha, b->alpha_tmp, x.n_tris, x.nobj, alpha,
                              n, per);
    if (rc) return rc;
    g_err.clear();
    return RR_OK;
}

int rr_batch_launch(rr_batch *b, void *const *cubes, int64_t *n_paths_out)
{
    if (!b || !cubes) return fail(RR_EINVAL, "NULL argument");
    for (int s = 0; s < b->S; s++)
        if (!cubes[s]) return fail(RR_EINVAL, "cube %d is NULL", s);
    rr_ctx *c = b->c;
    HIPCHK(hipSetDevice(c->device));
    bool new_cubes = b->cubes.size() != (size_t)b->S ||
                     !std::equal(b->cubes.begin(), b->cubes.end(), cubes);
    b->cubes.assign(cubes, cubes + b->S);
    // the exact engine's kernels take their cube as an argument: re-capture
    if (new_cubes && batch_any_freq(b)) b->dirty = true;
    for (int attempt = 0; attempt < 3; attempt++) {
        if (b->dirty || new_cubes) {
            int rc = batch_prepare(b);
            if (rc) return rc;
            new_cubes = false;
        }
        if (b->dirty) {
            // capture the whole pipeline once; later launches replay it
            batch_drop_graph(b);
            HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
            int rc = batch_enqueue_trace(b, false);
            if (!rc) rc = batch_enqueue_synth(b, false);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->st, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            HIPCHK(e);
            b->graph = g;
            HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            b->dirty = false;
        }
        HIPCHK(hipEventRecord(b->ev[4], c->stream));
        HIPCHK(hipStreamWaitEvent(b->st, b->ev[4], 0));
        HIPCHK(hipEventRecord(b->ev[0], b->st));
        HIPCHK(hipGraphLaunch(b->exec, b->st));
        HIPCHK(hipEventRecord(b->ev[5], b->st));
        HIPCHK(hipStreamWaitEvent(c->stream, b->ev[5], 0));
        bool overflow = false;
        int rc = batch_check(b, &overflow);
        if (rc) return rc;
        if (!overflow) break;
        b->dirty = true;
        if (attempt == 2) return fail(RR_EOVERFLOW, "batched path pool overflow persisted");
    }
    HIPCHK(hipEventElapsedTime(&b->ms_total, b->ev[0], b->ev[5]));
    if (n_paths_out)
        for (int s = 0; s < b->S; s++) n_paths_out[s] = b->sc[s].n_last;
    return RR_OK;
}

// paths per group timed for each tile candidate
static const int64_t TUNE_PATHS = 2048;

int rr_batch_tune(rr_batch *b, void *const *cubes)
{
    if (!b || !cubes) return fail(RR_EINVAL, "NULL argument");
    int rc = rr_batch_launch(b, cubes, nullptr);   // paths for the synthesis candidates
    if (rc) return rc;
    std::vector<int> Ks;
    for (auto &x : b->sc)
        if (std::find(Ks.begin(), Ks.end(), x.chirp.n_samples) == Ks.end()) Ks.push_back(x.chirp.n_samples);
    // the candidates run eagerly on a bounded prefix of the paths of the last
    // launch (time is linear in the path count)
    auto time_synth = [&](int only_K, int only_scene, float *ms) -> int {
        int r = batch_prepare(b, only_K, TUNE_PATHS, only_scene);
        if (r) return r;
        if ((r = batch_enqueue_synth(b, true))) return r;
        HIPCHK(hipStreamSynchronize(b->st));
        HIPCHK(hipEventElapsedTime(ms, b->ev[2], b->ev[3]));
        return RR_OK;
    };
    // 1. the direct engine's tile, per sample count, on every scene with it
    for (auto &x : b->sc) x.try_engine = RR_DIRECT_FP32;
    for (int K : Ks) {
        float best_ms = 3.0e38f;
        int best = 0;
        for (int cand : {32, 16, 8, 4}) {
            if (cand > RR_BATCH_MAX_KR || K % cand != 0 || K / cand > 256) continue;
            for (auto &x : b->sc)
                if (x.chirp.n_samples == K) x.kr = cand;
            float ms = 0.0f;
            if ((rc = time_synth(K, -1, &ms))) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = cand;
            }
        }
        if (rc) break;
        for (auto &x : b->sc)
            if (x.chirp.n_samples == K) x.kr = best;
    }
    // 2. per scene left to AUTO: the direct engine against the exact product
    // engine at each layout whose modelled cost is within 1.5x of the least
    // (in a per-element launch the Tx x Rx tiles waste the product on other
    // transmitters' rows and model accordingly).  The product engine's scene
    // runs as separate kernels: it has to win by a tenth and 20 us.
    for (int s = 0; s < b->S && !rc; s++) {
        BatchScene &x = b->sc[s];
        if (x.req_engine != RR_ENGINE_AUTO) continue;
        float t_direct = 0.0f;
        x.try_engine = RR_DIRECT_FP32;
        if ((rc = time_synth(0, s, &t_direct))) break;
        int best_eng = RR_DIRECT_FP32, best_tile = 0;
        float best_ms = t_direct;
        {
            const int K = x.chirp.n_samples;
            const bool pe = x.mode != RR_TX_SHARED;
            const double least = freq_tile_cost(x.ntx, x.nrx, K, freq_tile(x.ntx, x.nrx, K, pe), pe);
            for (int tile : {1, 16, 32, 48, 64, 96}) {
                if (freq_tile_cost(x.ntx, x.nrx, K, tile, pe) > 1.5 * least) continue;
                if (batch_freq_bytes(x, std::max(x.fq_cap, x.n_last), tile) > BATCH_FREQ_TABLE_MAX)
                    continue;
                x.try_engine = RR_GEMM_EXACT;
                x.try_tile = tile;
                float ms = 0.0f;
                if ((rc = time_synth(0, s, &ms))) break;
                if (ms * 1.1f + 0.02f < best_ms) {
                    best_ms = ms;
                    best_eng = RR_GEMM_EXACT;
                    best_tile = tile;
                }
            }
        }
        x.tuned_engine = best_eng;
        x.tuned_tile = best_tile;
    }
    for (auto &x : b->sc) x.try_engine = -1;
    batch_drop_graph(b);
    return rc;
}

int rr_batch_set_engine(rr_batch *b, int32_t slot, int32_t engine, int32_t tile)
{
    if (!b) return fail(RR_EINVAL, "NULL batch");
    if (slot < 0 || slot >= b->S) return fail(RR_EINVAL, "slot out of range");
    if (engine != RR_ENGINE_AUTO && engine != RR_DIRECT_FP32 && engine != RR_GEMM_EXACT)
        return fail(RR_EINVAL, "batched scenes use RR_ENGINE_AUTO, RR_DIRECT_FP32 or RR_GEMM_EXACT");
    if (tile != 0 && (engine != RR_GEMM_EXACT || (tile != 1 && tile != 16 && tile != 32 &&
                                                  tile != 48 && tile != 64 && tile != 96)))
        return fail(RR_EINVAL, "tile 1, 16, 32, 48, 64 or 96 with RR_GEMM_EXACT, else 0");
    if (tile == 1 && b->sc[slot].set && b->sc[slot].chirp.n_samples > 1024)
        return fail(RR_EINVAL, "the sample split takes at most 1024 samples");
    BatchScene &x = b->sc[slot];
    x.req_engine = engine;
    x.req_tile = tile;
    batch_drop_graph(b);
    return RR_OK;
}

int rr_batch_get_plan(rr_batch *b, int32_t *engine_out, int32_t *tile_out)
{
    if (!b || !engine_out || !tile_out) return fail(RR_EINVAL, "NULL argument");
    if (b->dirty) {
        HIPCHK(hipSetDevice(b->c->device));
        if (int rc = batch_prepare(b)) return rc;
    }
    for (int s = 0; s < b->S; s++) {
        BatchScene &x = b->sc[s];
        engine_out[s] = x.use_freq ? RR_GEMM_EXACT : RR_DIRECT_FP32;
        tile_out[s] = x.use_freq ? x.tile : x.kr;
    }
    return RR_OK;
}

int rr_batch_get_tiles(rr_batch *b, int32_t *kr_out)
{
    if (!b || !kr_out) return fail(RR_EINVAL, "NULL argument");
    for (int s = 0; s < b->S; s++) kr_out[s] = b->sc[s].kr;
    return RR_OK;
}

int rr_batch_stats(rr_batch *b, double *ms_total, double *ms_synth, int64_t *total_paths)
{
    if (!b) return fail(RR_EINVAL, "NULL argument");
    if (ms_total) *ms_total = b->ms_total;
    if (ms_synth) *ms_synth = b->ms_synth;
    if (total_paths) *total_paths = b->last_total;
    return RR_OK;
}

}  // extern "C"
