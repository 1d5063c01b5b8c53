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
// hi + lo bf16 parts (x = hi + lo to ~16 bits); each real product keeps
// hi*hi, hi*lo and lo*hi, accumulated in FP32.  The complex product uses
// three real products instead of four (Gauss's method, whose rounding Higham
// analysed in "Stability of a method for multiplying complex matrices with
// three real matrix multiplications", 1992):
//     P1 = Ar Br,  P2 = Ai Bi,  P3 = (Ar + Ai)(Br + Bi),
//     Re = P1 - P2,  Im = P3 - P1 - P2,
// so each 16-path step issues 9 MFMAs per 32x32 output block (12 with four
// real products), and both operands carry a third pair of planes for the
// sums Ar + Ai and Br + Bi, formed in FP32 before the split.
//
// A (channels x paths) is prepared once in the MFMA fragment layout, so a
// wavefront loads each 32x16 operand fragment as one contiguous 1 KiB read.
// B (paths x samples, up to 1.3e10 entries) is never stored: each workgroup
// generates its 16 x 64 tile per step into LDS from two 32-bit fixed-point
// phases per (path, chirp) -- start phase beta and per-sample step gamma,
// exact modulo 2^32 in integer arithmetic -- one hardware sin/cos per path
// and lane and a complex rotation by a precomputed exp(-j 2 pi 32 gamma).
#include "rr_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#define GM_TM 256          // output rows (channels) per workgroup
#define GM_TN 64           // output columns (chirp, sample) per workgroup
#define GM_KS 16           // paths per MFMA step
#define GM_THREADS 256     // 4 wavefronts, one per SIMD, 64 x 64 each
#define GM_WR 2            // 32-row blocks per wavefront
#define GM_NCB (GM_TN / 32)             // 32-column blocks per tile (each wavefront: all)
#define GM_PL 6            // operand planes: re hi, re lo, im hi, im lo, (re+im) hi, (re+im) lo
#define GM_NBUF 3          // B tiles in LDS: read one step ahead, generated two ahead
static_assert((GM_TM / 32 / GM_WR) == GM_THREADS / 64, "wavefront grid");
#define GM_BPAD 4          // padding after lane 31 of a B fragment in LDS (uint4 units)
#define BFRAG_U4 (64 + GM_BPAD)   // one B fragment in LDS (uint4 units)
#ifndef GM_VPM
#define GM_VPM 2           // vector instructions scheduled beside each MFMA
#endif


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
// uint4 index ((rb * KB + kb) * 6 + plane) * 64 + lane holds rows
// rb*32 + lane%32, paths kb*16 + (lane/32)*8 + 0..7 of plane
// (0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo, 4 (re+im)_hi, 5 (re+im)_lo).
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
    unsigned short h[GM_PL][8];
    // the lane's 8 paths of its Tx and Rx rows as four 16-byte loads each
    // (rows are Ppad = 96 k entries long, so every load is aligned)
    float4 ta[4], rb4[4];
    if (row < C) {
        const int t = row / nrx, r = row - t * nrx;
        const float4 *tp = reinterpret_cast<const float4 *>(T + (int64_t)t * Ppad + p0);
        const float4 *rp = reinterpret_cast<const float4 *>(R + (int64_t)r * Ppad + p0);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            ta[q] = tp[q];
            rb4[q] = rp[q];
        }
    }
#pragma unroll
    for (int e = 0; e < 8; e++) {
        float re = 0.0f, im = 0.0f;
        if (row < C) {
            const float4 av = ta[e >> 1], bv = rb4[e >> 1];
            const float2 a = (e & 1) ? make_float2(av.z, av.w) : make_float2(av.x, av.y);
            const float2 b = (e & 1) ? make_float2(bv.z, bv.w) : make_float2(bv.x, bv.y);
            re = a.x * b.x - a.y * b.y;
            im = a.x * b.y + a.y * b.x;
        }
        const float sm = re + im;
        unsigned short rh = bf16_bits(re), ih = bf16_bits(im), sh = bf16_bits(sm);
        h[0][e] = rh;
        h[1][e] = bf16_bits(re - bf16_float(rh));
        h[2][e] = ih;
        h[3][e] = bf16_bits(im - bf16_float(ih));
        h[4][e] = sh;
        h[5][e] = bf16_bits(sm - bf16_float(sh));
    }
    for (int q = 0; q < GM_PL; q++) {
        uint4 v;
        v.x = h[q][0] | ((unsigned)h[q][1] << 16);
        v.y = h[q][2] | ((unsigned)h[q][3] << 16);
        v.z = h[q][4] | ((unsigned)h[q][5] << 16);
        v.w = h[q][6] | ((unsigned)h[q][7] << 16);
        Af[(frag * GM_PL + q) * 64 + lane] = v;
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

// One workgroup computes a 256 x 64 output tile with four wavefronts, one
// per SIMD, stacked along the rows and each owning 64 x 64 (2 x 2 blocks of
// 32 x 32 with three accumulators each, P1, P2, P3: 192 accumulator
// registers).  Per 16-path step a wavefront issues 36 MFMAs.
//
// A fragments go from global memory (L2) straight into registers: each is
// one contiguous 1 KiB, and the six fragments of row block i for step kb + 2
// are requested as soon as the MFMAs of row block i of step kb have been
// issued (two register sets alternate).  B passes through LDS in three
// buffers, so one barrier per step suffices: in step kb a wavefront reads
// the fragments of B(kb + 1) into registers while the workgroup generates
// B(kb + 2); both are spread over the step's MFMAs.
__global__ __launch_bounds__(GM_THREADS, 1) void k_gemm(const uint4 *__restrict__ Af,
                                                        const uint4 *__restrict__ Bp, int RB,
                                                        int KB, int Ppad, int C, int M, int K,
                                                        int n_col_tiles, float2 *__restrict__ cube)
{
    // B: three buffers x 6 planes x column blocks, each fragment 64 lanes x
    // 16 B with 64 B of padding after lane 31, so that the generator's
    // 32-bit writes of both lane halves land in distinct banks (no bank
    // conflicts; with 128 B of padding a quarter of the LDS cycles were).
    __shared__ uint4 Bs[GM_NBUF][GM_PL * GM_NCB * BFRAG_U4];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // wavefront index, uniform by construction (kept in scalar registers)
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    // XCD-aware order: workgroup b runs on XCD b % 8; each XCD walks its own
    // contiguous run of (row tile, column tile) pairs, row tile slowest, so
    // the workgroups resident on one XCD share A through that XCD's L2.
    const int rtiles = RB / (GM_TM / 32);
    const int64_t total = (int64_t)rtiles * n_col_tiles;
    int64_t q = blockIdx.x;
    if (total % 8 == 0) q = (int64_t)(blockIdx.x % 8) * (total / 8) + blockIdx.x / 8;
    const int rt = (int)(q / n_col_tiles);
    const int ct = (int)(q - (int64_t)rt * n_col_tiles);
    const int rb0 = rt * (GM_TM / 32) + w * GM_WR;

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
    const int wofs = (flane * 16 + (flane >= 32 ? 16 * GM_BPAD : 0) + (p0 & 7) * 2) / 4;
    const uint4 *bprow = Bp + (int64_t)m * Ppad;   // + p0 per lane
    // words per plane (all column blocks)
    constexpr int PS = GM_NCB * BFRAG_U4 * 4;

    // generator state: the phasors of the two paths at the current column
    struct Gen {
        float ar, ai, br, bi, rar, rai, rbr, rbi;
    };
    // start phasors at column block 0 from the (beta, gamma) words
    auto gen_start = [&](uint4 pa, uint4 pb) -> Gen {
        Gen g;
        {
            const float u = (float)(int)(pa.x + kbase * pa.y) * 2.3283064365386963e-10f;
            g.ar = __builtin_amdgcn_cosf(u);
            g.ai = -__builtin_amdgcn_sinf(u);
        }
        {
            const float u = (float)(int)(pb.x + kbase * pb.y) * 2.3283064365386963e-10f;
            g.br = __builtin_amdgcn_cosf(u);
            g.bi = -__builtin_amdgcn_sinf(u);
        }
        g.rar = __uint_as_float(pa.z); g.rai = __uint_as_float(pa.w);
        g.rbr = __uint_as_float(pb.z); g.rbi = __uint_as_float(pb.w);
        return g;
    };
    // the six planes of column block h (after advancing by 32 columns for h > 0)
    auto gen_block = [&](Gen &g, int h, uint4 *B) {
        unsigned *bsw = reinterpret_cast<unsigned *>(B);
        if (h > 0) {
            float t0 = g.ar * g.rar - g.ai * g.rai, t1 = g.ar * g.rai + g.ai * g.rar;
            g.ar = t0; g.ai = t1;
            t0 = g.br * g.rbr - g.bi * g.rbi; t1 = g.br * g.rbi + g.bi * g.rbr;
            g.br = t0; g.bi = t1;
        }
        unsigned rh, rl, ih, il, sh, sl;
        split_bf16(g.ar, g.br, rh, rl);
        split_bf16(g.ai, g.bi, ih, il);
        split_bf16(g.ar + g.ai, g.br + g.bi, sh, sl);
        const int f = h * (BFRAG_U4 * 4) + wofs;
        bsw[f] = rh;
        bsw[f + PS] = rl;
        bsw[f + 2 * PS] = ih;
        bsw[f + 3 * PS] = il;
        bsw[f + 4 * PS] = sh;
        bsw[f + 5 * PS] = sl;
    };
    // A fragments of this wavefront's row blocks: fragment (rb, kb, plane)
    // is the 1 KiB at Af + ((rb KB + kb) 6 + plane) 64; the step's address is
    // uniform (scalar registers), the lane adds its own 16 bytes
    const uint4 *arow = Af + (int64_t)rb0 * KB * (GM_PL * 64);

    f32x16 p1[GM_WR][GM_NCB], p2[GM_WR][GM_NCB], p3[GM_WR][GM_NCB];
#pragma unroll
    for (int i = 0; i < GM_WR; i++)
#pragma unroll
        for (int j = 0; j < GM_NCB; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                p1[i][j][e] = 0.0f;
                p2[i][j][e] = 0.0f;
                p3[i][j][e] = 0.0f;
            }

    struct ARow {
        uint4 q[GM_PL];
    };
    struct BCols {
        uint4 q[GM_NCB][GM_PL];
    };
    auto load_a = [&](int kb, int i) -> ARow {
        ARow a;
        const uint4 *src = arow + ((int64_t)i * KB + kb) * (GM_PL * 64);
#pragma unroll
        for (int p = 0; p < GM_PL; p++) a.q[p] = src[p * 64 + lane];
        return a;
    };
    const int lofs = lane + (lane >= 32 ? GM_BPAD : 0);
    auto load_b = [&](const uint4 *B) -> BCols {
        BCols b;
#pragma unroll
        for (int j = 0; j < GM_NCB; j++)
#pragma unroll
            for (int p = 0; p < GM_PL; p++) b.q[j][p] = B[(p * GM_NCB + j) * BFRAG_U4 + lofs];
        return b;
    };
    // P1 += Ar Br, P2 += Ai Bi, P3 += (Ar + Ai)(Br + Bi), each hi*hi + hi*lo + lo*hi
    // (slot-major over both column blocks: consecutive MFMAs never share an
    // accumulator, the same one recurs every sixth)
    auto mma_row = [&](const ARow &a, const BCols &b, int i) {
#pragma unroll
        for (int s = 0; s < 3; s++) {
            const int ah = s == 2 ? 1 : 0, bl = s == 1 ? 1 : 0;   // hi*hi, hi*lo, lo*hi
#pragma unroll
            for (int j = 0; j < GM_NCB; j++) {
                p1[i][j] = MFMA(a.q[0 + ah], b.q[j][0 + bl], p1[i][j]);
                p2[i][j] = MFMA(a.q[2 + ah], b.q[j][2 + bl], p2[i][j]);
                p3[i][j] = MFMA(a.q[4 + ah], b.q[j][4 + bl], p3[i][j]);
            }
        }
    };

    // prologue: B(0) and B(1) in LDS, the B parameters of step 2 and the A
    // fragments of steps 0 and 1 in registers
    const int last = KB - 1;
    {
        Gen g0 = gen_start(bprow[p0], bprow[p0 + 1]);
#pragma unroll
        for (int h = 0; h < GM_NCB; h++) gen_block(g0, h, Bs[0]);
        const int s1 = min(1, last);
        Gen g1 = gen_start(bprow[(int64_t)s1 * GM_KS + p0], bprow[(int64_t)s1 * GM_KS + p0 + 1]);
#pragma unroll
        for (int h = 0; h < GM_NCB; h++) gen_block(g1, h, Bs[1]);
    }
    uint4 pna = bprow[(int64_t)min(2, last) * GM_KS + p0];
    uint4 pnb = bprow[(int64_t)min(2, last) * GM_KS + p0 + 1];
    ARow x0 = load_a(0, 0), x1 = load_a(0, 1);
    ARow y0 = load_a(min(1, last), 0), y1 = load_a(min(1, last), 1);
    __syncthreads();
    BCols b0 = load_b(Bs[0]), b1;

    // One step kb on A fragments r0, r1 (of step kb, loaded two steps
    // earlier) and B fragments bc; refills r0, r1 with step kb + 2, writes
    // B(kb + 2) into LDS and returns the B fragments of step kb + 1.
    auto step = [&](int kb, ARow &r0, ARow &r1, const BCols &bc, const uint4 *Br,
                    uint4 *Bg) -> BCols {
        const int nx = min(kb + 2, last);
        __syncthreads();        // B(kb + 1) complete; the buffer of B(kb + 2) is free
        BCols bn = load_b(Br);
        Gen g = gen_start(pna, pnb);
        // parameters of the next step's generation, a whole step ahead
        const int nb3 = min(kb + 3, last);
        pna = bprow[(int64_t)nb3 * GM_KS + p0];
        pnb = bprow[(int64_t)nb3 * GM_KS + p0 + 1];
        gen_block(g, 0, Bg);
        mma_row(r0, bc, 0);
#ifndef GM_FREE_SCHED
        __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);      // the two parameter loads
#pragma unroll
        for (int t = 0; t < 18; t++) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // 1 MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, GM_VPM, 0);  // GM_VPM VALU
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // up to 1 LDS read
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // up to 1 LDS write
        }
#endif
        __builtin_amdgcn_sched_barrier(0);
        r0 = load_a(nx, 0);
        gen_block(g, 1, Bg);
        mma_row(r1, bc, 1);
#ifndef GM_FREE_SCHED
#pragma unroll
        for (int t = 0; t < 18; t++) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // 1 MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, GM_VPM, 0);  // GM_VPM VALU
            __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // up to 1 LDS write
        }
#endif
        __builtin_amdgcn_sched_barrier(0);
        r1 = load_a(nx, 1);
        return bn;
    };
    // KB is a multiple of 6: the two A register sets and the three B buffers
    // return to the same places every six steps (constant LDS offsets)
    for (int kb = 0; kb < KB; kb += 6) {
        b1 = step(kb, x0, x1, b0, Bs[1], Bs[2]);
        b0 = step(kb + 1, y0, y1, b1, Bs[2], Bs[0]);
        b1 = step(kb + 2, x0, x1, b0, Bs[0], Bs[1]);
        b0 = step(kb + 3, y0, y1, b1, Bs[1], Bs[2]);
        b1 = step(kb + 4, x0, x1, b0, Bs[2], Bs[0]);
        b0 = step(kb + 5, y0, y1, b1, Bs[0], Bs[1]);
    }
    // Re = P1 - P2, Im = P3 - P1 - P2.  D layout: register e of lane l is
    // row 8*(e/4) + 4*(l/32) + e%4, column l%32
#pragma unroll
    for (int i = 0; i < GM_WR; i++)
#pragma unroll
        for (int j = 0; j < GM_NCB; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int row = (rb0 + i) * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
                const int k = k0 + j * 32 + (lane & 31);
                const float a = p1[i][j][e], b = p2[i][j][e];
                if (row < C && k < K)
                    cube[((int64_t)row * M + m) * K + k] = make_float2(a - b, p3[i][j][e] - a - b);
            }
}

}  // namespace

int gemm_row_pad() { return GM_TM; }
// bytes of the prepared A operand per (row, path): six bf16 planes
int gemm_a_bytes() { return 2 * GM_PL; }
int gemm_col_tile() { return GM_TN; }
// paths are padded to six steps (two A register sets, three B buffers)
int gemm_k_step() { return 6 * GM_KS; }

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
