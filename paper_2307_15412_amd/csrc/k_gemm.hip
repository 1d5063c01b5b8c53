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
    // B tile, two buffers x 4 planes x 4 column blocks x 64 lanes x 8 bf16
    __shared__ uint4 Bs[2][4][4][64];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
    // consecutive workgroups share a column tile (its B generation differs,
    // its A rows differ); the column tile changes slowest
    const int ct = blockIdx.x / (RB / (GM_TM / 32));
    const int rt = blockIdx.x - ct * (RB / (GM_TM / 32));
    const int64_t N = (int64_t)M * K;
    const int rb0 = rt * (GM_TM / 32) + wr * 2;

    // B generator: path row pl, base column nb; columns nb + 32 q, q = 0..3
    const int pl = tid >> 5;
    const int nb = tid & 31;
    const int64_t col0 = (int64_t)ct * GM_TN;
    const int m = (int)(col0 / K);
    const unsigned kbase = (unsigned)(col0 - (int64_t)m * K) + (unsigned)nb;
    const int flane = (pl >> 3) * 32 + nb;
    const int fslot = pl & 7;
    unsigned short *bsh = reinterpret_cast<unsigned short *>(&Bs[0][0][0][0]);

    auto gen = [&](int kb, int buf) {
        const uint4 prm = Bp[(int64_t)m * Ppad + (int64_t)kb * GM_KS + pl];
        const unsigned ph = prm.x + kbase * prm.y;
        const float u = (float)(int)ph * 2.3283064365386963e-10f;   // 2^-32, turns in [-1/2, 1/2)
        float zr = __builtin_amdgcn_cosf(u);
        float zi = -__builtin_amdgcn_sinf(u);
        const float rr = __uint_as_float(prm.z), ri = __uint_as_float(prm.w);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (q > 0) {
                float nr = zr * rr - zi * ri;
                float ni = zr * ri + zi * rr;
                zr = nr;
                zi = ni;
            }
            unsigned short rh = bf16_bits(zr), ih = bf16_bits(zi);
            unsigned short rl = bf16_bits(zr - bf16_float(rh));
            unsigned short il = bf16_bits(zi - bf16_float(ih));
            const int base = (((buf * 4 + 0) * 4 + q) * 64 + flane) * 8 + fslot;
            const int pstride = 4 * 64 * 8;
            bsh[base] = rh;
            bsh[base + pstride] = rl;
            bsh[base + 2 * pstride] = ih;
            bsh[base + 3 * pstride] = il;
        }
    };

    f32x16 sr[2][2], si[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) { sr[i][j][e] = 0.0f; si[i][j][e] = 0.0f; }

    gen(0, 0);
    __syncthreads();
    for (int kb = 0; kb < KB; kb++) {
        const int buf = kb & 1;
        uint4 a[2][4];
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int q = 0; q < 4; q++)
                a[i][q] = Af[(((int64_t)(rb0 + i) * KB + kb) * 4 + q) * 64 + lane];
        if (kb + 1 < KB) gen(kb + 1, buf ^ 1);
        uint4 b[2][4];
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int q = 0; q < 4; q++) b[j][q] = Bs[buf][q][wc * 2 + j][lane];
#pragma unroll
        for (int i = 0; i < 2; i++) {
            const uint4 nih = neg_bf(a[i][2]), nil = neg_bf(a[i][3]);
#pragma unroll
            for (int j = 0; j < 2; j++) {
                // re += Ar Br - Ai Bi ; im += Ar Bi + Ai Br  (hi*hi + hi*lo + lo*hi)
                sr[i][j] = MFMA(a[i][0], b[j][0], sr[i][j]);
                sr[i][j] = MFMA(a[i][0], b[j][1], sr[i][j]);
                sr[i][j] = MFMA(a[i][1], b[j][0], sr[i][j]);
                sr[i][j] = MFMA(nih, b[j][2], sr[i][j]);
                sr[i][j] = MFMA(nih, b[j][3], sr[i][j]);
                sr[i][j] = MFMA(nil, b[j][2], sr[i][j]);
                si[i][j] = MFMA(a[i][0], b[j][2], si[i][j]);
                si[i][j] = MFMA(a[i][0], b[j][3], si[i][j]);
                si[i][j] = MFMA(a[i][1], b[j][2], si[i][j]);
                si[i][j] = MFMA(a[i][2], b[j][0], si[i][j]);
                si[i][j] = MFMA(a[i][2], b[j][1], si[i][j]);
                si[i][j] = MFMA(a[i][3], b[j][0], si[i][j]);
            }
        }
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
