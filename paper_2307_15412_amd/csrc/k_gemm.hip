// k_gemm.hip -- cube synthesis as a complex GEMM on the gfx950 matrix cores.
//
// In the separable model the phase of path p in channel c = (t, r) at chirp
// m, sample k splits into a per-channel part and a per-(chirp, sample) part
// (Eq. 4 with the channel offsets of the path length taken at f0 and chirp 0):
//     s[c, n] = sum_p A[c, p] B[p, n],   n = m K + k,
//     A[c, p] = amp_p exp(-j 2 pi f0 (dT_p(t) + dR_p(r)) / c),
//     B[p, n] = exp(-j 2 pi (f0 + B k / K) D_p(m) / c).
// Phases are formed and reduced modulo one cycle in FP64 (prep kernels).  The
// GEMM runs in bf16 on v_mfma_f32_32x32x16_bf16 with each operand split into
// hi + lo bf16 parts (x = hi + lo to ~16 bits); the product keeps hi*hi,
// hi*lo and lo*hi, accumulated in FP32.  A complex product is four real ones,
// so each 16-path step issues 12 MFMAs per 32x32 output block.
//
// A (channels x paths) is prepared once in the MFMA fragment layout, so a
// wavefront loads each 32x16 operand fragment as one contiguous 1 KiB read.
// B (paths x samples, up to 1.3e10 entries) is never stored: each workgroup
// generates its 16 x 128 tile per step into LDS from two 32-bit fixed-point
// phases per (path, chirp) -- start phase beta and per-sample step gamma,
// exact modulo 2^32 in integer arithmetic -- one hardware sin/cos per lane
// and complex rotations by a precomputed exp(-j 2 pi 32 gamma).
#include "rr_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#define GM_TM 256          // output rows (channels) per workgroup
#define GM_TN 128          // output columns (chirp, sample) per workgroup
#define GM_KS 16           // paths per MFMA step
#define GM_THREADS 512     // 8 wavefronts: 4 (rows) x 2 (columns), 64 x 64 each
#define BFRAG_U4 72        // one B fragment in LDS: 64 lanes + 8 padding (uint4 units)

__device__ __forceinline__ double dist3(const double *a, const double *b)
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

__device__ __forceinline__ double frac(double x) { return x - floor(x); }

// exp(-j 2 pi u) for u in cycles, from the FP64-reduced phase
__device__ __forceinline__ float2 phasor64(double u)
{
    double f = frac(u);
    if (f >= 0.5) f -= 1.0;
    float s, c;
    sincospif(2.0f * (float)f, &s, &c);
    return make_float2(c, -s);
}

// T[t][p] (amp and Tx offset) and R[r][p] (Rx offset) at chirp 0
__global__ void k_prep_tr(SynthArgs A, int Ppad, float2 *T, float2 *R)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nT = (int64_t)A.ntx * Ppad, nR = (int64_t)A.nrx * Ppad;
    if (i >= nT + nR) return;
    const double f0c = A.f0 * A.inv_c;
    if (i < nT) {
        const int t = (int)(i / Ppad);
        const int64_t p = i - (int64_t)t * Ppad;
        float2 v = make_float2(0.0f, 0.0f);
        if (p < A.n_paths) {
            const SynPath &P = A.paths[p];
            if (P.src < 0 || P.src == t) {
                const double *os = P.src >= 0 ? A.tx + 3 * P.src : A.oT;
                const double dT = dist3(P.P[0], A.tx + 3 * t) - dist3(P.P[0], os);
                float2 z = phasor64(dT * f0c);
                const float a = (float)P.amp;
                v = make_float2(a * z.x, a * z.y);
            }
        }
        T[i] = v;
    } else {
        const int64_t j = i - nT;
        const int r = (int)(j / Ppad);
        const int64_t p = j - (int64_t)r * Ppad;
        float2 v = make_float2(0.0f, 0.0f);
        if (p < A.n_paths) {
            const SynPath &P = A.paths[p];
            const double *pk = P.P[P.K - 1];
            const double dR = dist3(A.rx + 3 * r, pk) - dist3(A.oR, pk);
            v = phasor64(dR * f0c);
        }
        R[j] = v;
    }
}

__device__ __forceinline__ unsigned short bf16_bits(float x)
{
    __bf16 h = (__bf16)x;
    return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_float(unsigned short b)
{
    return __builtin_bit_cast(float, (unsigned)b << 16);
}

// A[c][p] = T[t][p] R[r][p] split into bf16 hi/lo, in fragment order:
// uint4 index ((rb * KB + kb) * 4 + plane) * 64 + lane holds rows
// rb*32 + lane%32, paths kb*16 + (lane/32)*8 + 0..7 of plane
// (0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo).
__global__ void k_prep_a(const float2 *T, const float2 *R, int nrx, int C, int RB, int KB, int Ppad,
                         uint4 *Af)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)RB * KB * 64) return;
    const int lane = (int)(g & 63);
    const int64_t frag = g >> 6;
    const int kb = (int)(frag % KB);
    const int rb = (int)(frag / KB);
    const int row = rb * 32 + (lane & 31);
    const int64_t p0 = (int64_t)kb * GM_KS + (lane >> 5) * 8;
    unsigned short h[4][8];
    for (int e = 0; e < 8; e++) {
        float re = 0.0f, im = 0.0f;
        if (row < C) {
            const int t = row / nrx, r = row - (row / nrx) * nrx;
            float2 a = T[(int64_t)t * Ppad + p0 + e], b = R[(int64_t)r * Ppad + p0 + e];
            re = a.x * b.x - a.y * b.y;
            im = a.x * b.y + a.y * b.x;
        }
        unsigned short rh = bf16_bits(re), ih = bf16_bits(im);
        h[0][e] = rh;
        h[1][e] = bf16_bits(re - bf16_float(rh));
        h[2][e] = ih;
        h[3][e] = bf16_bits(im - bf16_float(ih));
    }
    for (int q = 0; q < 4; q++) {
        uint4 v;
        v.x = h[q][0] | ((unsigned)h[q][1] << 16);
        v.y = h[q][2] | ((unsigned)h[q][3] << 16);
        v.z = h[q][4] | ((unsigned)h[q][5] << 16);
        v.w = h[q][6] | ((unsigned)h[q][7] << 16);
        Af[(frag * 4 + q) * 64 + lane] = v;
    }
}

// Per (chirp m, path p): beta = frac(f0 D / c), gamma = frac(B D / (K c)) as
// 32-bit fixed point, and exp(-j 2 pi 64 gamma) for the column rotation.
__global__ void k_prep_b(SynthArgs A, int Ppad, uint4 *Bp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)A.M * Ppad) return;
    const int m = (int)(i / Ppad);
    const int64_t p = i - (int64_t)m * Ppad;
    uint4 out = make_uint4(0u, 0u, __float_as_uint(1.0f), 0u);
    if (p < A.n_paths) {
        const SynPath &P = A.paths[p];
        const double tau = (double)m * A.t_rep;
        double q1[3], qk[3];
        for (int a = 0; a < 3; a++) q1[a] = P.P[0][a] + P.V[0][a] * tau;
        double inner = 0.0;
        for (int a = 0; a < 3; a++) qk[a] = q1[a];
        for (int j = 1; j < P.K; j++) {
            double q[3];
            for (int a = 0; a < 3; a++) q[a] = P.P[j][a] + P.V[j][a] * tau;
            inner += dist3(q, qk);
            for (int a = 0; a < 3; a++) qk[a] = q[a];
        }
        const double *os = P.src >= 0 ? A.tx + 3 * P.src : A.oT;
        const double D = dist3(q1, os) + inner + dist3(A.oR, qk);
        const double beta = frac(D * A.f0 * A.inv_c);
        const double gamma = frac(D * (A.bw / (double)A.K) * A.inv_c);
        const double two32 = 4294967296.0;
        out.x = (unsigned)(unsigned long long)llrint(beta * two32);
        out.y = (unsigned)(unsigned long long)llrint(gamma * two32);
        float2 z = phasor64(64.0 * gamma);
        out.z = __float_as_uint(z.x);
        out.w = __float_as_uint(z.y);
    }
    Bp[i] = out;
}

__device__ __forceinline__ bf16x8 as_bf(uint4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ uint4 neg_bf(uint4 v)
{
    return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

#define MFMA(a, b, c) __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(a), as_bf(b), c, 0, 0, 0)

__global__ __launch_bounds__(GM_THREADS, 1) void k_gemm(const uint4 *__restrict__ Af,
                                                        const uint4 *__restrict__ Bp, int RB,
                                                        int KB, int Ppad, int C, int M, int K,
                                                        int n_col_tiles, float2 *__restrict__ cube)
{
    // A tile: two buffers x 8 row blocks x 4 planes x 64 lanes (uint4 = 8 bf16).
    // B tile: two buffers x 4 planes x 4 column blocks, each fragment 64 lanes
    // x 16 B with 128 B of padding after lane 31, so that the generator's
    // 32-bit writes of both lane halves land in distinct banks.
    __shared__ uint4 As[2][GM_TM / 32][4][64];
    __shared__ uint4 Bs[2 * 4 * 4 * BFRAG_U4];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    // XCD-aware order: workgroup b runs on XCD b % 8; each XCD walks its own
    // contiguous run of (row tile, column tile) pairs, row tile slowest, so
    // the workgroups resident on one XCD share A through that XCD's L2.
    const int rtiles = RB / (GM_TM / 32);
    const int64_t total = (int64_t)rtiles * n_col_tiles;
    int64_t q = blockIdx.x;
    if (total % 8 == 0) q = (int64_t)(blockIdx.x % 8) * (total / 8) + blockIdx.x / 8;
    const int rt = (int)(q / n_col_tiles);
    const int ct = (int)(q - (int64_t)rt * n_col_tiles);
    const int64_t N = (int64_t)M * K;
    const int rb0 = rt * (GM_TM / 32) + wr * 2;

    // B generator: path pair (2 pp, 2 pp + 1), columns nb and nb + 64 of the tile
    const int pp = tid & 7;
    const int nb = tid >> 3;
    const int64_t col0 = (int64_t)ct * GM_TN;
    const int m = (int)(col0 / K);
    const unsigned kbase = (unsigned)(col0 - (int64_t)m * K) + (unsigned)nb;
    const int p0 = 2 * pp;
    const int flane = (p0 >> 3) * 32 + (nb & 31);
    // 32-bit word index of (fragment 0, this lane, slots p0 & 7 and +1)
    const int wofs = (flane * 16 + (flane >= 32 ? 128 : 0) + (p0 & 7) * 2) / 4;
    unsigned *bsw = reinterpret_cast<unsigned *>(Bs);
    const uint4 *bprow = Bp + (int64_t)m * Ppad + p0;

    auto gen = [&](uint4 pa, uint4 pb, int buf) {
        // start phasors of both paths at column nb, then rotate by 64 columns
        float ar, ai, br, bi;
        {
            const float u = (float)(int)(pa.x + kbase * pa.y) * 2.3283064365386963e-10f;
            ar = __builtin_amdgcn_cosf(u);
            ai = -__builtin_amdgcn_sinf(u);
        }
        {
            const float u = (float)(int)(pb.x + kbase * pb.y) * 2.3283064365386963e-10f;
            br = __builtin_amdgcn_cosf(u);
            bi = -__builtin_amdgcn_sinf(u);
        }
#pragma unroll
        for (int h = 0; h < 2; h++) {
            if (h == 1) {
                const float rar = __uint_as_float(pa.z), rai = __uint_as_float(pa.w);
                const float rbr = __uint_as_float(pb.z), rbi = __uint_as_float(pb.w);
                float t0 = ar * rar - ai * rai, t1 = ar * rai + ai * rar;
                ar = t0; ai = t1;
                t0 = br * rbr - bi * rbi; t1 = br * rbi + bi * rbr;
                br = t0; bi = t1;
            }
            const unsigned rh = bf16_bits(ar) | ((unsigned)bf16_bits(br) << 16);
            const unsigned ih = bf16_bits(ai) | ((unsigned)bf16_bits(bi) << 16);
            const unsigned rl = bf16_bits(ar - bf16_float((unsigned short)rh)) |
                                ((unsigned)bf16_bits(br - bf16_float((unsigned short)(rh >> 16))) << 16);
            const unsigned il = bf16_bits(ai - bf16_float((unsigned short)ih)) |
                                ((unsigned)bf16_bits(bi - bf16_float((unsigned short)(ih >> 16))) << 16);
            const int cb = (nb >> 5) + 2 * h;
            // word offset of (buf, plane, column block cb)
            const int f = ((buf * 4 + 0) * 4 + cb) * (BFRAG_U4 * 4);
            const int ps = 4 * BFRAG_U4 * 4;
            bsw[f + wofs] = rh;
            bsw[f + ps + wofs] = rl;
            bsw[f + 2 * ps + wofs] = ih;
            bsw[f + 3 * ps + wofs] = il;
        }
    };
    // A staging: the tile of one step is 8 row blocks x 4 planes x 64 lanes;
    // thread tid moves entries tid + 512 r, r = 0..3 (1 KiB contiguous runs)
    const uint4 *abase = Af + (int64_t)rt * (GM_TM / 32) * KB * 256;
    // (staged values travel by value in a struct so that they stay in VGPRs)
    struct Stage {
        uint4 r0, r1, r2, r3;
    };
    const int rbl0 = tid >> 8, rest0 = tid & 255;
    auto stage_load = [&](int kb) -> Stage {
        Stage v;
        const uint4 *src = abase + (int64_t)kb * 256 + rest0;
        const int64_t rstride = (int64_t)KB * 256;
        v.r0 = src[(int64_t)(rbl0 + 0) * rstride];
        v.r1 = src[(int64_t)(rbl0 + 2) * rstride];
        v.r2 = src[(int64_t)(rbl0 + 4) * rstride];
        v.r3 = src[(int64_t)(rbl0 + 6) * rstride];
        return v;
    };
    auto stage_store = [&](const Stage v, int buf) {
        uint4 *dst = &As[buf][0][0][0] + tid;
        dst[0] = v.r0;
        dst[GM_THREADS] = v.r1;
        dst[2 * GM_THREADS] = v.r2;
        dst[3 * GM_THREADS] = v.r3;
    };

    f32x16 sr[2][2], si[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) { sr[i][j][e] = 0.0f; si[i][j][e] = 0.0f; }

    struct Frags {
        uint4 a[2][4], b[2][4];
    };
    auto load_frags = [&](int buf) -> Frags {
        Frags f;
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int q = 0; q < 4; q++) f.a[i][q] = As[buf][wr * 2 + i][q][lane];
        const int lofs = lane + (lane >= 32 ? 8 : 0);
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int q = 0; q < 4; q++)
                f.b[j][q] = Bs[((buf * 4 + q) * 4 + wc * 2 + j) * BFRAG_U4 + lofs];
        return f;
    };
    auto mma = [&](const Frags &f) {
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const uint4 nih = neg_bf(f.a[i][2]), nil = neg_bf(f.a[i][3]);
#pragma unroll
            for (int j = 0; j < 2; j++) {
                // re += Ar Br - Ai Bi ; im += Ar Bi + Ai Br  (hi*hi + hi*lo + lo*hi)
                sr[i][j] = MFMA(f.a[i][0], f.b[j][0], sr[i][j]);
                si[i][j] = MFMA(f.a[i][0], f.b[j][2], si[i][j]);
                sr[i][j] = MFMA(f.a[i][0], f.b[j][1], sr[i][j]);
                si[i][j] = MFMA(f.a[i][0], f.b[j][3], si[i][j]);
                sr[i][j] = MFMA(f.a[i][1], f.b[j][0], sr[i][j]);
                si[i][j] = MFMA(f.a[i][1], f.b[j][2], si[i][j]);
                sr[i][j] = MFMA(nih, f.b[j][2], sr[i][j]);
                si[i][j] = MFMA(f.a[i][2], f.b[j][0], si[i][j]);
                sr[i][j] = MFMA(nih, f.b[j][3], sr[i][j]);
                si[i][j] = MFMA(f.a[i][2], f.b[j][1], si[i][j]);
                sr[i][j] = MFMA(nil, f.b[j][2], sr[i][j]);
                si[i][j] = MFMA(f.a[i][3], f.b[j][0], si[i][j]);
            }
        }
    };

    // Pipeline: the global loads of step kb + 2 are issued during step kb and
    // only written to LDS at the start of step kb + 1, a full step later, so
    // their latency hides behind one step of matrix-core work.  Indices are
    // clamped instead of branched; the surplus work at the end fills the LDS
    // buffer that is no longer read.
    const int last = KB - 1;
    Stage v = stage_load(0);
    stage_store(v, 0);
    gen(bprow[0], bprow[1], 0);
    v = stage_load(min(1, last));
    uint4 pna = bprow[(int64_t)min(1, last) * GM_KS];
    uint4 pnb = bprow[(int64_t)min(1, last) * GM_KS + 1];
    __syncthreads();
    for (int kb = 0; kb < KB; kb++) {
        const int buf = kb & 1;
        stage_store(v, buf ^ 1);
        const int nx = min(kb + 2, last);
        const uint4 pca = pna, pcb = pnb;
        v = stage_load(nx);
        pna = bprow[(int64_t)nx * GM_KS];
        pnb = bprow[(int64_t)nx * GM_KS + 1];
        // keep the prefetch loads above the matrix-core work
        __builtin_amdgcn_sched_barrier(0);
        const Frags f = load_frags(buf);
        gen(pca, pcb, buf ^ 1);
        mma(f);
        // interleave the generation of the next B tile (VALU, LDS writes)
        // with this step's MFMAs so that the matrix cores stay busy
        __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);   // fragment reads
#pragma unroll
        for (int g = 0; g < 8; g++) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // 1 MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);  // 6 VALU
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // 1 LDS write
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 40, 0);
        __syncthreads();
    }
    // D layout: register e of lane l is row 8*(e/4) + 4*(l/32) + e%4, column l%32
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int row = (rb0 + i) * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const int64_t col = col0 + (wc * 2 + j) * 32 + (lane & 31);
                if (row < C) cube[(int64_t)row * N + col] = make_float2(sr[i][j][e], si[i][j][e]);
            }
}

}  // namespace

int gemm_row_pad() { return GM_TM; }
int gemm_col_tile() { return GM_TN; }
int gemm_k_step() { return GM_KS; }

hipError_t launch_gemm_prep_tr(const SynthArgs &a, int Ppad, float2 *T, float2 *R, hipStream_t s)
{
    const int64_t n = (int64_t)(a.ntx + a.nrx) * Ppad;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep_tr, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, Ppad, T, R);
    return hipGetLastError();
}

hipError_t launch_gemm_prep_a(const float2 *T, const float2 *R, int nrx, int C, int Cpad, int Ppad,
                              uint4 *Af, hipStream_t s)
{
    const int RB = Cpad / 32, KB = Ppad / GM_KS;
    const int64_t n = (int64_t)RB * KB * 64;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep_a, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T, R, nrx, C,
                       RB, KB, Ppad, Af);
    return hipGetLastError();
}

hipError_t launch_gemm_prep_b(const SynthArgs &a, int Ppad, uint4 *Bp, hipStream_t s)
{
    const int64_t n = (int64_t)a.M * Ppad;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep_b, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, Ppad, Bp);
    return hipGetLastError();
}

hipError_t launch_gemm_main(const uint4 *Af, const uint4 *Bp, int Cpad, int Ppad, int C, int M,
                            int K, float2 *cube, hipStream_t s)
{
    const int RB = Cpad / 32, KB = Ppad / GM_KS;
    const int64_t N = (int64_t)M * K;
    const int64_t n_col_tiles = N / GM_TN;
    const int64_t blocks = (int64_t)(Cpad / GM_TM) * n_col_tiles;
    if (blocks <= 0 || KB <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gemm, dim3((unsigned)blocks), dim3(GM_THREADS), 0, s, Af, Bp, RB, KB, Ppad,
                       C, M, K, (int)n_col_tiles, cube);
    return hipGetLastError();
}
