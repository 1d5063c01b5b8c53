// k_synth.hip -- direct coherent summation of received paths into the FMCW
// beat-signal cube (Section III-B, Eq. 4, with the stepped frequency replaced
// by the chirp's instantaneous frequency f_k = f0 + B k / K).
//
// Each lane owns one (channel, chirp) row and a run of KR consecutive fast-time
// samples.  Paths are staged through LDS in chunks.  For every (path, row) of
// the chunk the workgroup forms the path length once, in FP64, and reduces
// the carrier phase f0 d / c and the per-sample step B d / (K c) modulo one
// cycle in FP64 (the phase at 77 GHz is ~1e4 cycles, beyond FP32), keeping
// both as 32-bit fixed-point turns in an LDS table.  A lane then forms the
// start phase of its run exactly in integer arithmetic (beta + k0 gamma modulo
// 2^32), takes the hardware sin/cos of it and of the step (input in turns),
// and walks the run by complex rotation, accumulating in FP32 registers.  A
// second kernel evaluates individual cube entries fully in FP64 for checks at
// sizes where the whole cube is not needed.
#include <algorithm>

#include "rr_internal.h"

namespace {

#define SYN_T 256
#define SYN_CHUNK 32
#define SYN_TAB 4096      // (path, row) phase entries per chunk: 32 KiB of LDS

__device__ __forceinline__ double dist3(double ax, double ay, double az, double bx, double by,
                                        double bz)
{
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// Per (path, channel, chirp): lengths such that the phase of sample k is
//   phi_k = d_base * f0 / c + k * d_step * B / (K c)   (cycles).
// Exact model: d_base = d_step = |p_1(m) - tx_t| + inner(m) + |rx_r - p_K(m)|.
// Separable model: d_step = D(m) = |p_1(m) - o_s| + inner(m) + |o_R - p_K(m)|
// and d_base = D(m) + dT + dR with the channel offsets dT, dR taken at chirp 0.
__device__ __forceinline__ void path_lengths(const SynthArgs &A, const SynPath &P, double tau,
                                             const double *tx, const double *rx, double &d_base,
                                             double &d_step)
{
    const int K = P.K;
    double x1 = P.P[0][0] + P.V[0][0] * tau, y1 = P.P[0][1] + P.V[0][1] * tau,
           z1 = P.P[0][2] + P.V[0][2] * tau;
    double xk = x1, yk = y1, zk = z1;
    double inner = 0.0;
    for (int j = 1; j < K; j++) {
        double x = P.P[j][0] + P.V[j][0] * tau, y = P.P[j][1] + P.V[j][1] * tau,
               z = P.P[j][2] + P.V[j][2] * tau;
        inner += dist3(x, y, z, xk, yk, zk);
        xk = x; yk = y; zk = z;
    }
    if (A.model == RR_EXACT) {
        double d = dist3(x1, y1, z1, tx[0], tx[1], tx[2]) + inner +
                   dist3(rx[0], rx[1], rx[2], xk, yk, zk);
        d_base = d;
        d_step = d;
    } else {
        double os[3];
        if (P.src >= 0) {
            os[0] = A.tx[3 * P.src]; os[1] = A.tx[3 * P.src + 1]; os[2] = A.tx[3 * P.src + 2];
        } else {
            os[0] = A.oT[0]; os[1] = A.oT[1]; os[2] = A.oT[2];
        }
        const double *p1 = P.P[0], *pk = P.P[K - 1];
        double dT = dist3(p1[0], p1[1], p1[2], tx[0], tx[1], tx[2]) -
                    dist3(p1[0], p1[1], p1[2], os[0], os[1], os[2]);
        double dR = dist3(rx[0], rx[1], rx[2], pk[0], pk[1], pk[2]) -
                    dist3(A.oR[0], A.oR[1], A.oR[2], pk[0], pk[1], pk[2]);
        double D = dist3(x1, y1, z1, os[0], os[1], os[2]) + inner +
                   dist3(A.oR[0], A.oR[1], A.oR[2], xk, yk, zk);
        d_base = D + (dT + dR);
        d_step = D;
    }
}

__device__ __forceinline__ double frac(double x) { return x - floor(x); }

// x modulo one cycle as 32-bit fixed-point turns
__device__ __forceinline__ unsigned turns_u32(double x)
{
    return (unsigned)(unsigned long long)llrint(frac(x) * 4294967296.0);
}

// fixed-point turns -> FP32 turns in [-1/2, 1/2)
__device__ __forceinline__ float turns_f32(unsigned u)
{
    return (float)(int)u * 2.3283064365386963e-10f;
}

// One workgroup tile: rows rb * RPB .. of group g (a Tx in the per-element
// mode, everything in the shared mode), every sample of those rows.
template <int KR>
__device__ void synth_block(const SynthArgs &A, int g, int rb, int rows_per_group, int RC,
                            SynPath *sp, uint2 *tab)
{
    const int TPR = A.K / KR;
    const int RPB = SYN_T / TPR;
    const int lrow = threadIdx.x / TPR;
    const int row = rb * RPB + lrow;
    const int k0 = (threadIdx.x % TPR) * KR;
    const bool valid = lrow < RPB && row < rows_per_group;
    const double f0c = A.f0 * A.inv_c;
    const double bkc = A.bw / (double)A.K * A.inv_c;
    float are[KR], aim[KR];
#pragma unroll
    for (int k = 0; k < KR; k++) { are[k] = 0.0f; aim[k] = 0.0f; }
    const int64_t p0 = A.ranges[g];
    const int64_t p1 = A.p_limit > 0 ? min(A.ranges[g + 1], p0 + A.p_limit) : A.ranges[g + 1];
    const int chunk = min(SYN_CHUNK, SYN_TAB / RPB);
    for (int64_t base = p0; base < p1; base += chunk) {
        const int cnt = (int)min((int64_t)chunk, p1 - base);
        __syncthreads();
        {
            const float4 *srcv = reinterpret_cast<const float4 *>(A.paths + base);
            float4 *dstv = reinterpret_cast<float4 *>(sp);
            const int nv = cnt * (int)(sizeof(SynPath) / sizeof(float4));
            for (int i = threadIdx.x; i < nv; i += SYN_T) dstv[i] = srcv[i];
        }
        __syncthreads();
        // phase table, entry q * RPB + l: (beta, gamma) of path q in row l
        for (int e = threadIdx.x; e < cnt * RPB; e += SYN_T) {
            const int q = e / RPB, l = e - q * RPB;
            const int rw = rb * RPB + l;
            uint2 v = make_uint2(0u, 0u);
            if (rw < rows_per_group) {
                const int m = rw / RC, cc = rw - (rw / RC) * RC;
                const int c = A.shared ? cc : g * A.nrx + cc;
                const int t = c / A.nrx, r = c - (c / A.nrx) * A.nrx;
                const double tx[3] = {A.tx[3 * t], A.tx[3 * t + 1], A.tx[3 * t + 2]};
                const double rx[3] = {A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]};
                double db, ds;
                path_lengths(A, sp[q], (double)m * A.t_rep, tx, rx, db, ds);
                v = make_uint2(turns_u32(db * f0c), turns_u32(ds * bkc));
            }
            tab[e] = v;
        }
        __syncthreads();
        if (!valid) continue;
        for (int q = 0; q < cnt; q++) {
            const uint2 ph = tab[q * RPB + lrow];
            const float a = (float)sp[q].amp;
            // exp(-j 2 pi phi) = cos - j sin, phi in turns
            const float u0 = turns_f32(ph.x + (unsigned)k0 * ph.y);
            const float u1 = turns_f32(ph.y);
            float pr = a * __builtin_amdgcn_cosf(u0), pi = -a * __builtin_amdgcn_sinf(u0);
            const float rr = __builtin_amdgcn_cosf(u1), ri = -__builtin_amdgcn_sinf(u1);
#pragma unroll
            for (int k = 0; k < KR; k++) {
                are[k] += pr;
                aim[k] += pi;
                float nr = pr * rr - pi * ri;
                float ni = pr * ri + pi * rr;
                pr = nr;
                pi = ni;
            }
        }
    }
    if (!valid) return;
    const int m = row / RC, cc = row - (row / RC) * RC;
    const int c = A.shared ? cc : g * A.nrx + cc;
    float2 *out = A.cube + ((int64_t)c * A.M + m) * A.K + k0;
#pragma unroll
    for (int k = 0; k < KR; k++) out[k] = make_float2(are[k], aim[k]);
}

template <int KR>
__global__ __launch_bounds__(SYN_T) void k_synth_direct(SynthArgs A, int rows_per_group, int RC,
                                                        int blocks_per_group)
{
    __shared__ SynPath sp[SYN_CHUNK];
    __shared__ uint2 tab[SYN_TAB];
    const int g = blockIdx.x / blocks_per_group;
    synth_block<KR>(A, g, blockIdx.x - g * blocks_per_group, rows_per_group, RC, sp, tab);
}

// Batched, persistent: workgroups pull (scene, tile) items from a device
// counter; each scene carries its own tile shape (samples per lane KR, chosen
// by the autotuner) and its path range comes from the batched scan.
__global__ __launch_bounds__(SYN_T) void k_batch_synth(const SynthArgs *scenes,
                                                       const BatchSynthInfo *info,
                                                       const int64_t *item_start, int S,
                                                       unsigned long long *work)
{
    __shared__ SynPath sp[SYN_CHUNK];
    __shared__ uint2 tab[SYN_TAB];
    __shared__ long long s_item;
    const int64_t n_items = item_start[S];
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (long long)atomicAdd(work, 1ull);
        __syncthreads();
        // the item is the same in every lane: keep it, the scene search and
        // the scene's arguments in scalar registers
        const long long iv = s_item;
        const int64_t it = (int64_t)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                                          (int)(iv >> 32)) << 32) |
                                     (unsigned)__builtin_amdgcn_readfirstlane((int)iv));
        if (it >= n_items) break;
        int lo = 0, hi = S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (item_start[mid] <= it) lo = mid; else hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const SynthArgs A = scenes[lo];
        const BatchSynthInfo I = info[lo];
        const int local = (int)(it - item_start[lo]);
        const int g = local / I.bpg;
        const int rb = local - g * I.bpg;
        switch (I.kr) {
#if RR_BATCH_MAX_KR >= 32
        case 32: synth_block<32>(A, g, rb, I.rows_per_group, I.rc, sp, tab); break;
#endif
        case 16: synth_block<16>(A, g, rb, I.rows_per_group, I.rc, sp, tab); break;
        case 8: synth_block<8>(A, g, rb, I.rows_per_group, I.rc, sp, tab); break;
        case 4: synth_block<4>(A, g, rb, I.rows_per_group, I.rc, sp, tab); break;
        case 2: synth_block<2>(A, g, rb, I.rows_per_group, I.rc, sp, tab); break;
        default: synth_block<1>(A, g, rb, I.rows_per_group, I.rc, sp, tab); break;
        }
    }
}

// one block per requested entry; FP64 phase, FP64 sin/cos, FP64 accumulation
__global__ __launch_bounds__(256) void k_synth_sampled(SynthArgs A, const int64_t *idx)
{
    __shared__ double sre[256], sim[256];
    const int64_t f = idx[blockIdx.x];
    const int64_t MK = (int64_t)A.M * A.K;
    if (f < 0 || f >= (int64_t)(A.ntx * A.nrx) * MK) {
        if (threadIdx.x == 0) A.cube[blockIdx.x] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
        return;
    }
    const int c = (int)(f / MK);
    const int m = (int)((f / A.K) % A.M);
    const int k = (int)(f % A.K);
    const int t = c / A.nrx, r = c % A.nrx;
    const double tx[3] = {A.tx[3 * t], A.tx[3 * t + 1], A.tx[3 * t + 2]};
    const double rx[3] = {A.rx[3 * r], A.rx[3 * r + 1], A.rx[3 * r + 2]};
    const double tau = (double)m * A.t_rep;
    const double fk = A.f0 + A.bw * (double)k / (double)A.K;
    const int64_t p0 = A.shared ? 0 : A.ranges[t], p1 = A.shared ? A.n_paths : A.ranges[t + 1];
    double re = 0.0, im = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
        const SynPath &P = A.paths[p];
        double db, ds;
        path_lengths(A, P, tau, tx, rx, db, ds);
        double phase = (A.f0 * db + (fk - A.f0) * ds) * A.inv_c;
        double fr = frac(phase);
        double s, cs;
        sincospi(2.0 * fr, &s, &cs);
        re += P.amp * cs;
        im -= P.amp * s;
    }
    sre[threadIdx.x] = re;
    sim[threadIdx.x] = im;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sre[threadIdx.x] += sre[threadIdx.x + off];
            sim[threadIdx.x] += sim[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) A.cube[blockIdx.x] = make_float2((float)sre[0], (float)sim[0]);
}

__global__ void k_syn_prep(PathSoA P, int64_t n, const double *obj_vel, int nobj,
                           const double *pt_vel, int npts, SynPath *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    SynPath s;
    const int64_t cap = P.cap;
#pragma unroll
    for (int q = 0; q < RR_KMAX; q++) {
        int vid = P.vid[q * cap + i];
        const double *v = nullptr;
        if (vid >= 0 && vid < nobj) v = obj_vel + 3 * vid;
        else if (vid >= nobj && vid < nobj + npts) v = pt_vel + 3 * (vid - nobj);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            s.P[q][a] = P.p[(3 * q + a) * cap + i];
            s.V[q][a] = v ? v[a] : 0.0;
        }
    }
    s.amp = P.amp[i];
    s.K = P.K[i];
    s.src = P.src[i];
    out[i] = s;
}

// ranges[g] = first path with src >= g (paths sorted by src); g in [0, n_groups]
// ranges[g] = first path whose source is >= g0 + g, g = 0 .. n_groups (src
// sorted): per-Tx groups with g0 = 0, the single group of a shared launch
// (every src = -1) with g0 = -1
__global__ void k_ranges(const int32_t *src, int64_t n, int n_groups, int g0, int64_t *ranges)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > n_groups) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (src[mid] < g0 + g) lo = mid + 1; else hi = mid;
    }
    ranges[g] = lo;
}

// synthesis records of the batched path pool: the scene of a path follows
// from its virtual ray id
__global__ void k_batch_prep(PathSoA P, const unsigned long long *total, int64_t cap,
                             const int64_t *vr_start, int S, const BatchVel *vel, SynPath *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = min((int64_t)*total, cap);
    if (i >= n) return;
    const int64_t v = P.ray[i];
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (vr_start[mid] <= v) lo = mid; else hi = mid - 1;
    }
    const BatchVel &bv = vel[lo];
    SynPath s;
    const int64_t c = P.cap;
#pragma unroll
    for (int q = 0; q < RR_KMAX; q++) {
        const int vid = P.vid[q * c + i];
        const double *vv = nullptr;
        if (vid >= 0 && vid < bv.nobj) vv = bv.obj_vel + 3 * vid;
        else if (vid >= bv.nobj && vid < bv.nobj + bv.npts) vv = bv.pt_vel + 3 * (vid - bv.nobj);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            s.P[q][a] = P.p[(3 * q + a) * c + i];
            s.V[q][a] = vv ? vv[a] : 0.0;
        }
    }
    s.amp = P.amp[i];
    s.K = P.K[i];
    s.src = P.src[i];
    out[i] = s;
}

// per-scene path ranges from the batched exclusive scan: paths of virtual
// rays [vr0 + t n_vps, ...) start at offsets[vr0 + t n_vps]
__global__ void k_batch_ranges(const uint32_t *offsets, int64_t V, const unsigned long long *total,
                               int64_t cap, const BatchRangeInfo *ri, int S, int64_t *ranges)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const BatchRangeInfo &R = ri[s];
    const int64_t tot = min((int64_t)*total, cap);
    auto off = [&](int64_t v) -> int64_t {
        const int64_t o = v < V ? (int64_t)offsets[v] : tot;
        return min(o, tot);
    };
    if (R.shared) {
        ranges[R.base] = off(R.vr0);
        ranges[R.base + 1] = off(R.vr0 + R.n_vps);
    } else {
        for (int g = 0; g <= R.n_groups; g++) ranges[R.base + g] = off(R.vr0 + (int64_t)g * R.n_vps);
    }
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_batch_synth(const SynthArgs *scenes, const BatchSynthInfo *info,
                              const int64_t *item_start, int S, int64_t n_items,
                              unsigned long long *work, hipStream_t s)
{
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t grid = std::min<int64_t>(n_items, (int64_t)cus * 8);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_synth, dim3((unsigned)grid), dim3(SYN_T), 0, s, scenes, info,
                       item_start, S, work);
    return hipGetLastError();
}

hipError_t launch_batch_prep(const PathSoA &paths, const unsigned long long *total, int64_t cap,
                             const int64_t *vr_start, int S, const BatchVel *vel, SynPath *out,
                             hipStream_t s)
{
    if (cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, paths,
                       total, cap, vr_start, S, vel, out);
    return hipGetLastError();
}

hipError_t launch_batch_ranges(const uint32_t *offsets, int64_t V, const unsigned long long *total,
                               int64_t cap, const BatchRangeInfo *ri, int S, int64_t *ranges,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_ranges, dim3((unsigned)((S + 63) / 64)), dim3(64), 0, s, offsets, V,
                       total, cap, ri, S, ranges);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_syn_prep(const PathSoA &paths, int64_t n, const double *obj_vel, int nobj,
                           const double *pt_vel, int npts, SynPath *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_syn_prep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, paths, n,
                       obj_vel, nobj, pt_vel, npts, out);
    return hipGetLastError();
}

hipError_t launch_ranges(const int32_t *src, int64_t n, int n_groups, int g0, int64_t *ranges,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((n_groups + 1 + 255) / 256)), dim3(256), 0, s,
                       src, n, n_groups, g0, ranges);
    return hipGetLastError();
}

template <int KR>
static hipError_t launch_kr(const SynthArgs &a, int n_groups, int rows_per_group, int RC,
                            hipStream_t s)
{
    const int TPR = a.K / KR;
    const int RPB = SYN_T / TPR;
    const int bpg = (rows_per_group + RPB - 1) / RPB;
    const int64_t blocks = (int64_t)bpg * n_groups;
    hipLaunchKernelGGL(k_synth_direct<KR>, dim3((unsigned)blocks), dim3(SYN_T), 0, s, a,
                       rows_per_group, RC, bpg);
    return hipGetLastError();
}

hipError_t launch_synth_direct(const SynthArgs &a, int n_groups, int rows_per_group,
                               hipStream_t s)
{
    const int RC = a.shared ? a.ntx * a.nrx : a.nrx;
    int kr = 32;
    while (kr > 1 && a.K % kr != 0) kr >>= 1;
    if (a.K / kr > SYN_T) return hipErrorInvalidValue;
    switch (kr) {
    case 32: return launch_kr<32>(a, n_groups, rows_per_group, RC, s);
    case 16: return launch_kr<16>(a, n_groups, rows_per_group, RC, s);
    case 8: return launch_kr<8>(a, n_groups, rows_per_group, RC, s);
    case 4: return launch_kr<4>(a, n_groups, rows_per_group, RC, s);
    case 2: return launch_kr<2>(a, n_groups, rows_per_group, RC, s);
    default: return launch_kr<1>(a, n_groups, rows_per_group, RC, s);
    }
}

hipError_t launch_synth_sampled(const SynthArgs &a, const int64_t *idx, int64_t n_idx,
                                hipStream_t s)
{
    if (n_idx <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_synth_sampled, dim3((unsigned)n_idx), dim3(256), 0, s, a, idx);
    return hipGetLastError();
}
