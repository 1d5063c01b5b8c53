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
// exact modulo 2^32 in integer arithmetic -- one hardware sin/cos per path
// and lane and complex rotations by a precomputed exp(-j 2 pi 32 gamma).
#include "rr_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#ifndef GM_TM
#define GM_TM 512          // output rows (channels) per workgroup
#endif
#ifndef GM_TN
#define GM_TN 64           // output columns (chirp, sample) per workgroup
#endif
#define GM_KS 16           // paths per MFMA step
#define GM_THREADS 256     // 4 wavefronts, one per SIMD, 128 x 64 each
#define GM_WR 4            // 32-row blocks per wavefront
#define GM_WC 2            // 32-column blocks per wavefront
#define GM_NCB (GM_TN / 32)             // column blocks per tile
#define GM_WAVES_C (GM_NCB / GM_WC)     // wavefronts across the columns
static_assert((GM_TM / 32 / GM_WR) * GM_WAVES_C == GM_THREADS / 64, "wavefront grid");
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
// 32-bit fixed point, and exp(-j 2 pi 32 gamma) for the column rotation.
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
        float2 z = phasor64(32.0 * gamma);
        out.z = __float_as_uint(z.x);
        out.w = __float_as_uint(z.y);
    }
    Bp[i] = out;
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// (x, y) -> packed bf16 (x low, y high), round to nearest even
__device__ __forceinline__ unsigned pack_bf16(float x, float y)
{
    f32x2 v = {x, y};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}
// hi = bf16(x, y); lo = bf16(x - hi.x, y - hi.y): x = hi + lo to ~16 bits
__device__ __forceinline__ void split_bf16(float x, float y, unsigned &hi, unsigned &lo)
{
    hi = pack_bf16(x, y);
    lo = pack_bf16(x - __uint_as_float(hi << 16), y - __uint_as_float(hi & 0xffff0000u));
}

__device__ __forceinline__ bf16x8 as_bf(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

#define MFMA(a, b, c) __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(a), as_bf(b), c, 0, 0, 0)

// One workgroup computes a 512 x 64 output tile with four wavefronts, one
// per SIMD, stacked along the rows and each owning 128 x 64 (4 x 2 blocks of
// 32 x 32, accumulators in the AGPR half of the register file).  Per 16-path
// step a wavefront issues 96 MFMAs.  The tall tile shares each generated B
// value among 512 rows and gives every A fragment to exactly one wavefront.
//
// A fragments go from global memory (L2) straight into registers: each is
// one contiguous 1 KiB, and the fragments of row block i for step kb + 2 are
// requested as soon as the MFMAs of row i of step kb have been issued, two
// steps before they are needed (two register sets alternate).  Only B passes through LDS (two buffers):
//   first half of step kb: MFMAs of rows 0-1, interleaved with the
//     generation of B(kb + 1);
//   barrier (B(kb + 1) complete);
//   second half: MFMAs of rows 2-3 while the B fragments of step kb + 1 are
//     read into registers.
__global__ __launch_bounds__(GM_THREADS, 1) void k_gemm(const uint4 *__restrict__ Af,
                                                        const uint4 *__restrict__ Bp, int RB,
                                                        int KB, int Ppad, int C, int M, int K,
                                                        int n_col_tiles, float2 *__restrict__ cube)
{
    // B: two buffers x 4 planes (re_hi, re_lo, im_hi, im_lo) x column blocks,
    // each fragment 64 lanes x 16 B with 128 B of padding after lane 31, so
    // that the generator's 32-bit writes of both lane halves land in distinct
    // banks.
    __shared__ uint4 Bs[2][4 * GM_NCB * BFRAG_U4];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // wavefront index, uniform by construction (kept in scalar registers)
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = w / GM_WAVES_C, wc = w % GM_WAVES_C;
    // XCD-aware order: workgroup b runs on XCD b % 8; each XCD walks its own
    // contiguous run of (row tile, column tile) pairs, row tile slowest, so
    // the workgroups resident on one XCD share A through that XCD's L2.
    const int rtiles = RB / (GM_TM / 32);
    const int64_t total = (int64_t)rtiles * n_col_tiles;
    int64_t q = blockIdx.x;
    if (total % 8 == 0) q = (int64_t)(blockIdx.x % 8) * (total / 8) + blockIdx.x / 8;
    const int rt = (int)(q / n_col_tiles);
    const int ct = (int)(q - (int64_t)rt * n_col_tiles);
    const int rb0 = rt * (GM_TM / 32) + wr * GM_WR;

    // B generator: path pair (2 pp, 2 pp + 1), columns nb + 32 h, h < GM_NCB
    const int pp = tid & 7;
    const int nb = tid >> 3;
    // column tile ct: chirp m, samples k0 .. k0 + GM_TN - 1 (each chirp's
    // samples are padded to whole tiles; samples k >= K are not stored)
    const int tpc = (K + GM_TN - 1) / GM_TN;
    const int m = ct / tpc;
    const int k0 = (ct - m * tpc) * GM_TN;
    const unsigned kbase = (unsigned)k0 + (unsigned)nb;
    const int p0 = 2 * pp;
    const int flane = (p0 >> 3) * 32 + nb;
    // 32-bit word index of (fragment 0, this lane, slots p0 & 7 and +1)
    const int wofs = (flane * 16 + (flane >= 32 ? 128 : 0) + (p0 & 7) * 2) / 4;
    const uint4 *bprow = Bp + (int64_t)m * Ppad + p0;

    auto gen = [&](uint4 pa, uint4 pb, uint4 *Bs) {
        unsigned *bsw = reinterpret_cast<unsigned *>(Bs);
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
        const float rar = __uint_as_float(pa.z), rai = __uint_as_float(pa.w);
        const float rbr = __uint_as_float(pb.z), rbi = __uint_as_float(pb.w);
#pragma unroll
        for (int h = 0; h < GM_NCB; h++) {
            if (h > 0) {
                // advance both phasors by 32 columns
                float t0 = ar * rar - ai * rai, t1 = ar * rai + ai * rar;
                ar = t0; ai = t1;
                t0 = br * rbr - bi * rbi; t1 = br * rbi + bi * rbr;
                br = t0; bi = t1;
            }
            unsigned rh, rl, ih, il;
            split_bf16(ar, br, rh, rl);
            split_bf16(ai, bi, ih, il);
            // word offset of (plane 0, column block h)
            const int f = h * (BFRAG_U4 * 4);
            const int ps = GM_NCB * BFRAG_U4 * 4;
            bsw[f + wofs] = rh;
            bsw[f + ps + wofs] = rl;
            bsw[f + 2 * ps + wofs] = ih;
            bsw[f + 3 * ps + wofs] = il;
        }
    };
    // A fragments of this wavefront's row blocks: fragment (rb, kb, plane)
    // is the 1 KiB at Af + ((rb KB + kb) 4 + plane) 64
    const uint4 *arow = Af + (int64_t)rb0 * KB * 256 + lane;

    f32x16 sr[GM_WR][GM_WC], si[GM_WR][GM_WC];
#pragma unroll
    for (int i = 0; i < GM_WR; i++)
#pragma unroll
        for (int j = 0; j < GM_WC; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) { sr[i][j][e] = 0.0f; si[i][j][e] = 0.0f; }

    struct ARow {
        uint4 q[4];
    };
    // B fragments of two column blocks: planes (re_hi, re_lo, im_hi, im_lo)
    // in q, the negated imaginary planes for the real part of the product in n
    struct BCols {
        uint4 q[GM_WC][4];
        uint4 n[GM_WC][2];
    };
    auto load_a = [&](int kb, int i) -> ARow {
        ARow a;
        const uint4 *src = arow + ((int64_t)i * KB + kb) * 256;
#pragma unroll
        for (int p = 0; p < 4; p++) a.q[p] = src[p * 64];
        return a;
    };
    const int lofs = lane + (lane >= 32 ? 8 : 0);
    auto load_b = [&](const uint4 *Bs) -> BCols {
        BCols b;
#pragma unroll
        for (int j = 0; j < GM_WC; j++)
#pragma unroll
            for (int p = 0; p < 4; p++) b.q[j][p] = Bs[(p * GM_NCB + wc * GM_WC + j) * BFRAG_U4 + lofs];
        return b;
    };
    // sign flip of the imaginary planes (bf16 negation is exact); applied
    // well after the LDS reads, so that it never waits for them
    auto negate = [&](BCols &b) {
#pragma unroll
        for (int j = 0; j < GM_WC; j++)
#pragma unroll
            for (int p = 0; p < 2; p++) {
                const uint4 v = b.q[j][2 + p];
                b.n[j][p] = make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u,
                                       v.w ^ 0x80008000u);
            }
    };
    // re += Ar Br + Ai (-Bi) ; im += Ar Bi + Ai Br  (hi*hi + hi*lo + lo*hi)
    auto mma_row = [&](const ARow a, const BCols &b, int i) {
#pragma unroll
        for (int j = 0; j < GM_WC; j++) {
            sr[i][j] = MFMA(a.q[0], b.q[j][0], sr[i][j]);
            si[i][j] = MFMA(a.q[0], b.q[j][2], si[i][j]);
            sr[i][j] = MFMA(a.q[0], b.q[j][1], sr[i][j]);
            si[i][j] = MFMA(a.q[0], b.q[j][3], si[i][j]);
            sr[i][j] = MFMA(a.q[1], b.q[j][0], sr[i][j]);
            si[i][j] = MFMA(a.q[1], b.q[j][2], si[i][j]);
            sr[i][j] = MFMA(a.q[2], b.n[j][0], sr[i][j]);
            si[i][j] = MFMA(a.q[2], b.q[j][0], si[i][j]);
            sr[i][j] = MFMA(a.q[2], b.n[j][1], sr[i][j]);
            si[i][j] = MFMA(a.q[2], b.q[j][1], si[i][j]);
            sr[i][j] = MFMA(a.q[3], b.n[j][0], sr[i][j]);
            si[i][j] = MFMA(a.q[3], b.q[j][0], si[i][j]);
        }
    };

    // prologue: B(0) in LDS, the B parameters of step 1 and the A fragments
    // of steps 0 and 1 in registers
    const int last = KB - 1;
    gen(bprow[0], bprow[1], Bs[0]);
    uint4 pna = bprow[(int64_t)min(1, last) * GM_KS];
    uint4 pnb = bprow[(int64_t)min(1, last) * GM_KS + 1];
    ARow x0 = load_a(0, 0), x1 = load_a(0, 1), x2 = load_a(0, 2), x3 = load_a(0, 3);
    ARow y0 = load_a(min(1, last), 0), y1 = load_a(min(1, last), 1);
    ARow y2 = load_a(min(1, last), 2), y3 = load_a(min(1, last), 3);
    __syncthreads();
    BCols b0 = load_b(Bs[0]), b1;
    negate(b0);

    // One step kb on A fragments r0..r3 (of step kb, loaded two steps
    // earlier) and B fragments bc; refills r0..r3 with step kb + 2 and
    // returns the B fragments of step kb + 1.
    auto step = [&](int kb, ARow &r0, ARow &r1, ARow &r2, ARow &r3, const BCols &bc) -> BCols {
        const int nx = min(kb + 2, last);
        uint4 *Bn = Bs[(kb + 1) & 1];
        const uint4 pca = pna, pcb = pnb;
        // rows 0-1 with the generation of B(kb + 1) interleaved
        gen(pca, pcb, Bn);
        mma_row(r0, bc, 0);
#ifndef GM_FREE_SCHED
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
#pragma unroll
        for (int g = 0; g < 16; g++) {
            __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // 3 VALU
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // up to 1 LDS write
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // 1 MFMA
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 23 - 16, 0);
#endif
        __builtin_amdgcn_sched_barrier(0);
        r0 = load_a(nx, 0);
        pna = bprow[(int64_t)nx * GM_KS];
        pnb = bprow[(int64_t)nx * GM_KS + 1];
        mma_row(r1, bc, 1);
        __builtin_amdgcn_sched_barrier(0);
        r1 = load_a(nx, 1);
        __syncthreads();
        BCols bn = load_b(Bn);
        mma_row(r2, bc, 2);
        __builtin_amdgcn_sched_barrier(0);
        r2 = load_a(nx, 2);
        negate(bn);
        mma_row(r3, bc, 3);
        __builtin_amdgcn_sched_barrier(0);
        r3 = load_a(nx, 3);
        return bn;
    };
    // KB is even: the two register sets alternate
    for (int kb = 0; kb < KB; kb += 2) {
        b1 = step(kb, x0, x1, x2, x3, b0);
        b0 = step(kb + 1, y0, y1, y2, y3, b1);
    }
    // D layout: register e of lane l is row 8*(e/4) + 4*(l/32) + e%4, column l%32
#pragma unroll
    for (int i = 0; i < GM_WR; i++)
#pragma unroll
        for (int j = 0; j < GM_WC; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int row = (rb0 + i) * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const int k = k0 + (wc * GM_WC + j) * 32 + (lane & 31);
                if (row < C && k < K)
                    cube[((int64_t)row * M + m) * K + k] = make_float2(sr[i][j][e], si[i][j][e]);
            }
}

}  // namespace

int gemm_row_pad() { return GM_TM; }
int gemm_col_tile() { return GM_TN; }
// paths are padded to two steps (the A register sets alternate)
int gemm_k_step() { return 2 * GM_KS; }

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
    const int64_t n_col_tiles = (int64_t)M * ((K + GM_TN - 1) / GM_TN);
    const int64_t blocks = (int64_t)(Cpad / GM_TM) * n_col_tiles;
    if (n_col_tiles > INT32_MAX || blocks > UINT32_MAX) return hipErrorInvalidValue;
    if (blocks <= 0 || KB <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gemm, dim3((unsigned)blocks), dim3(GM_THREADS), 0, s, Af, Bp, RB, KB, Ppad,
                       C, M, K, (int)n_col_tiles, cube);
    return hipGetLastError();
}
