// k_freq.hip -- exact-model synthesis (Eq. 4, every path length in full) as
// one complex matrix product per (chirp, sample) on the matrix cores.
//
// The path length of channel (t, r) splits exactly into a Tx part and an Rx
// part, d = dX(t) + dY(r) with dX = |p_1(m) - tx_t| + inner(m) and
// dY = |rx_r - p_K(m)|, so for every chirp m and sample k
//     s[t, r, m, k] = sum_p X[t, p] Y[p, r],
//     X[t, p] = a_p exp(-j 2 pi f_k dX / c),   Y[p, r] = exp(-j 2 pi f_k dY / c),
// with f_k = f0 + B k / K: a (Tx x paths) by (paths x Rx) complex product, the
// same multiply-adds as the direct sum but on MFMA.  No approximation is made
// (unlike the separable model); a path of the per-element launch has
// X[t, p] = 0 for every t other than its own transmitter.
//
// Both legs are reduced in FP64 per (chirp, element, path) to 32-bit
// fixed-point turns: beta = frac(f0 d / c), gamma = frac(B d / (K c)), so the
// phase at sample k is beta + k gamma modulo 2^32, exact in integer
// arithmetic.  A workgroup of three wavefronts computes a 96 x 96 (Tx x Rx)
// output tile of one (chirp, sample) over one split of the paths, 16 paths per
// step: each wavefront generates its own 32 rows of X straight into A-operand
// registers, the three together generate the 16 x 96 Y tile into LDS (double
// buffered), and each wavefront issues 36 v_mfma_f32_32x32x16_bf16 per step.
// Operands are split bf16 hi + lo, products hi*hi + hi*lo + lo*hi, FP32
// accumulation (as the separable GEMM).  Several path splits write partial
// tiles that a second kernel adds in split order (deterministic).
#include "rr_internal.h"

namespace {

#define FQ_W 3            // wavefronts per workgroup (32 Tx rows each)
#define FQ_TILE 96        // Tx and Rx extent of a workgroup tile
#define FQ_KS 16          // paths per step

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ double frac(double x) { return x - floor(x); }

__device__ __forceinline__ unsigned turns_u32(double x)
{
    return (unsigned)(unsigned long long)llrint(frac(x) * 4294967296.0);
}

__device__ __forceinline__ double dist3(const double *a, const double *b)
{
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// Per (chirp, path): first and last hit point at chirp time and the length
// between them.  Layout [M][Ppad] of 8 doubles: p1.xyz, pK.xyz, inner, amp.
__global__ void k_freq_paths(const SynPath *paths, int64_t n, int64_t Ppad, int M, double t_rep,
                             double *pm)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)M * Ppad) return;
    const int m = (int)(g / Ppad);
    const int64_t p = g - (int64_t)m * Ppad;
    double *o = pm + 8 * g;
    if (p >= n) {
        for (int q = 0; q < 8; q++) o[q] = 0.0;
        return;
    }
    const SynPath &P = paths[p];
    const double tau = (double)m * t_rep;
    double q1[3], qk[3], inner = 0.0;
    for (int a = 0; a < 3; a++) q1[a] = P.P[0][a] + P.V[0][a] * tau;
    for (int a = 0; a < 3; a++) qk[a] = q1[a];
    for (int j = 1; j < P.K; j++) {
        double q[3];
        for (int a = 0; a < 3; a++) q[a] = P.P[j][a] + P.V[j][a] * tau;
        inner += dist3(q, qk);
        for (int a = 0; a < 3; a++) qk[a] = q[a];
    }
    for (int a = 0; a < 3; a++) {
        o[a] = q1[a];
        o[3 + a] = qk[a];
    }
    o[6] = inner;
    o[7] = P.amp;
}

// Leg tables: xt[m][t][p] for dX = |p1 - tx_t| + inner and yt[m][r][p] for
// dY = |rx_r - pK|, each (beta, gamma) in fixed-point turns; and per path the
// amplitude (0 beyond the path count) and source.
__global__ void k_freq_tables(const double *pm, const SynPath *paths, int64_t n, int64_t Ppad, int M,
                              const double *tx, int T, const double *rx, int R, double f0c,
                              double dfc, uint2 *xt, uint2 *yt, float *amp, int32_t *src)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_m = (int64_t)(T + R) * Ppad;
    if (g >= (int64_t)M * per_m) return;
    const int m = (int)(g / per_m);
    const int64_t rem = g - (int64_t)m * per_m;
    const int i = (int)(rem / Ppad);
    const int64_t p = rem - (int64_t)i * Ppad;
    const double *o = pm + 8 * ((int64_t)m * Ppad + p);
    uint2 v = make_uint2(0u, 0u);
    if (p < n) {
        const double d = i < T ? dist3(o, tx + 3 * i) + o[6] : dist3(rx + 3 * (i - T), o + 3);
        v = make_uint2(turns_u32(d * f0c), turns_u32(d * dfc));
    }
    if (i < T)
        xt[((int64_t)m * T + i) * Ppad + p] = v;
    else
        yt[((int64_t)m * R + (i - T)) * Ppad + p] = v;
    if (m == 0 && i == 0) {
        amp[p] = p < n ? (float)paths[p].amp : 0.0f;
        src[p] = p < n ? paths[p].src : -1;
    }
}

__device__ __forceinline__ unsigned pack_bf16(float x, float y)
{
    f32x2 v = {x, y};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

// hi = bf16(x, y); lo = bf16(x - hi.x, y - hi.y)
__device__ __forceinline__ void split_bf16(float x, float y, unsigned &hi, unsigned &lo)
{
    hi = pack_bf16(x, y);
    lo = pack_bf16(x - __uint_as_float(hi << 16), y - __uint_as_float(hi & 0xffff0000u));
}

__device__ __forceinline__ bf16x8 as_bf(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

#define MFMA(a, b, c) __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(a), as_bf(b), c, 0, 0, 0)

// exp(-j 2 pi u) of fixed-point turns u
__device__ __forceinline__ void phasor(unsigned u, float &re, float &im)
{
    const float f = (float)(int)u * 2.3283064365386963e-10f;
    re = __builtin_amdgcn_cosf(f);
    im = -__builtin_amdgcn_sinf(f);
}

struct Frag {          // one 32 x 16 operand, split: real hi/lo, imaginary hi/lo
    uint4 rh, rl, ih, il;
};

struct Raw {           // one lane's table words of one step: 8 (beta, gamma) pairs
    uint4 w[4];
};

__device__ __forceinline__ Raw load_raw(const uint2 *row)
{
    const uint4 *r4 = reinterpret_cast<const uint4 *>(row);
    Raw r;
#pragma unroll
    for (int q = 0; q < 4; q++) r.w[q] = r4[q];
    return r;
}

// the 8 path slots of one fragment lane at sample k, times a (when given),
// split into the four bf16 planes
__device__ __forceinline__ Frag leg_frag(const Raw &raw, unsigned k, const float *a)
{
    const unsigned *wv = reinterpret_cast<const unsigned *>(raw.w);
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
        phasor(wv[2 * e] + k * wv[2 * e + 1], re[e], im[e]);
        if (a) {
            re[e] *= a[e];
            im[e] *= a[e];
        }
    }
    Frag f;
    unsigned *rh = &f.rh.x, *rl = &f.rl.x, *ih = &f.ih.x, *il = &f.il.x;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        split_bf16(re[2 * q], re[2 * q + 1], rh[q], rl[q]);
        split_bf16(im[2 * q], im[2 * q + 1], ih[q], il[q]);
    }
    return f;
}

__device__ __forceinline__ uint4 neg(uint4 v)
{
    return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

struct FreqArgs {
    const uint2 *xt, *yt;
    const float *amp;
    const int32_t *src;
    int T, R, M, K;
    int64_t Ppad;
    int tt, rt;               // Tx and Rx tiles
    int n_split;
    int64_t split_len;        // paths per split (multiple of FQ_KS)
    float2 *out;              // cube (one split) or partial tiles [split][m][k][T][R]
    int partial;
};

__global__ __launch_bounds__(FQ_W * 64) void k_freq_gemm(FreqArgs A)
{
    __shared__ uint4 Ys[2][FQ_W][4][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // k fastest: the workgroups that share one split's tables run together
    int64_t id = blockIdx.x;
    const int k = (int)(id % A.K);
    id /= A.K;
    const int ri = (int)(id % A.rt);
    id /= A.rt;
    const int ti = (int)(id % A.tt);
    id /= A.tt;
    const int m = (int)(id % A.M);
    const int s = (int)(id / A.M);
    const int64_t pbeg = (int64_t)s * A.split_len;
    const int64_t pend = min(A.Ppad, pbeg + A.split_len);
    const int t = ti * FQ_TILE + w * 32 + (lane & 31);
    const int ry = ri * FQ_TILE + w * 32 + (lane & 31);   // Rx row this lane generates
    const int half = (lane >> 5) * 8;
    const bool tv = t < A.T, rv = ry < A.R;
    const uint2 *xrow = A.xt + ((int64_t)m * A.T + (tv ? t : 0)) * A.Ppad + half;
    const uint2 *yrow = A.yt + ((int64_t)m * A.R + (rv ? ry : 0)) * A.Ppad + half;
    const unsigned ku = (unsigned)k;

    // per step and lane: the X and Y table words of its 8 path slots and
    // those paths' amplitudes (masked for other transmitters in the
    // per-element launch), loaded one step ahead of their use
    struct Step {
        Raw x, y;
        float a[8];
    };
    auto load = [&](int64_t p0) -> Step {
        Step st;
        st.x = load_raw(xrow + p0);
        st.y = load_raw(yrow + p0);
        const float4 *a4 = reinterpret_cast<const float4 *>(A.amp + p0 + half);
        const int4 *s4 = reinterpret_cast<const int4 *>(A.src + p0 + half);
        const float4 a0 = a4[0], a1 = a4[1];
        const int4 s0 = s4[0], s1 = s4[1];
        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const int sv[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
        for (int e = 0; e < 8; e++) st.a[e] = (tv && (sv[e] < 0 || sv[e] == t)) ? av[e] : 0.0f;
        return st;
    };
    auto put_y = [&](const Raw &raw, int buf) {
        Frag f = leg_frag(raw, ku, nullptr);
        if (!rv) f.rh = f.rl = f.ih = f.il = make_uint4(0u, 0u, 0u, 0u);
        Ys[buf][w][0][lane] = f.rh;
        Ys[buf][w][1][lane] = f.rl;
        Ys[buf][w][2][lane] = f.ih;
        Ys[buf][w][3][lane] = f.il;
    };

    f32x16 sr[FQ_W], si[FQ_W];
#pragma unroll
    for (int j = 0; j < FQ_W; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) {
            sr[j][e] = 0.0f;
            si[j][e] = 0.0f;
        }
    // table words two steps ahead of their use (the leg tables stream from
    // beyond L2; one step of products does not cover that latency)
    Step cur = load(pbeg);
    Step nx1 = load(pbeg + FQ_KS < pend ? pbeg + FQ_KS : pbeg);
    Frag x = leg_frag(cur.x, ku, cur.a);
    put_y(cur.y, 0);
    __syncthreads();
    int buf = 0;
    for (int64_t p0 = pbeg; p0 < pend; p0 += FQ_KS) {
        const bool more = p0 + FQ_KS < pend;
        const int64_t p2 = p0 + 2 * FQ_KS < pend ? p0 + 2 * FQ_KS : p0;
        Step nx2 = load(p2);
        uint4 y[FQ_W][4];
#pragma unroll
        for (int j = 0; j < FQ_W; j++)
#pragma unroll
            for (int q = 0; q < 4; q++) y[j][q] = Ys[buf][j][q][lane];
        const uint4 nih = neg(x.ih), nil = neg(x.il);
#pragma unroll
        for (int j = 0; j < FQ_W; j++) {
            // re += Xr Yr - Xi Yi, im += Xr Yi + Xi Yr (each hi*hi + hi*lo + lo*hi)
            sr[j] = MFMA(x.rh, y[j][0], sr[j]);
            sr[j] = MFMA(x.rh, y[j][1], sr[j]);
            sr[j] = MFMA(x.rl, y[j][0], sr[j]);
            sr[j] = MFMA(nih, y[j][2], sr[j]);
            sr[j] = MFMA(nih, y[j][3], sr[j]);
            sr[j] = MFMA(nil, y[j][2], sr[j]);
            si[j] = MFMA(x.rh, y[j][2], si[j]);
            si[j] = MFMA(x.rh, y[j][3], si[j]);
            si[j] = MFMA(x.rl, y[j][2], si[j]);
            si[j] = MFMA(x.ih, y[j][0], si[j]);
            si[j] = MFMA(x.ih, y[j][1], si[j]);
            si[j] = MFMA(x.il, y[j][0], si[j]);
        }
        if (more) {
            put_y(nx1.y, buf ^ 1);
            x = leg_frag(nx1.x, ku, nx1.a);
        }
        nx1 = nx2;
        buf ^= 1;
        __syncthreads();
    }
    // D layout: register e of lane l is row 8 (e / 4) + 4 (l / 32) + e % 4
    // (a Tx row of this wavefront's block), column l % 32 (an Rx column)
#pragma unroll
    for (int j = 0; j < FQ_W; j++)
#pragma unroll
        for (int e = 0; e < 16; e++) {
            const int to = ti * FQ_TILE + w * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
            const int ro = ri * FQ_TILE + j * 32 + (lane & 31);
            if (to < A.T && ro < A.R) {
                const float2 v = make_float2(sr[j][e], si[j][e]);
                if (A.partial)
                    A.out[((((int64_t)s * A.M + m) * A.K + k) * A.T + to) * A.R + ro] = v;
                else
                    A.out[(((int64_t)to * A.R + ro) * A.M + m) * A.K + k] = v;
            }
        }
}

// cube[(t R + r) M + m][k] = sum over splits, in split order
__global__ void k_freq_reduce(const float2 *part, int n_split, int T, int R, int M, int K,
                              float2 *cube)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)M * K * T * R;
    if (g >= per) return;
    // g enumerates (m, k, t, r) with r fastest: coalesced partial reads
    const int r = (int)(g % R);
    int64_t q = g / R;
    const int t = (int)(q % T);
    q /= T;
    const int k = (int)(q % K);
    const int m = (int)(q / K);
    float re = 0.0f, im = 0.0f;
    for (int s = 0; s < n_split; s++) {
        const float2 v = part[(int64_t)s * per + g];
        re += v.x;
        im += v.y;
    }
    cube[(((int64_t)t * R + r) * M + m) * K + k] = make_float2(re, im);
}

}  // namespace

int freq_k_step() { return FQ_KS; }

hipError_t launch_freq_prep(const SynPath *paths, int64_t n, int64_t Ppad, int M, double t_rep,
                            const double *tx, int T, const double *rx, int R, double f0c, double dfc,
                            double *pm, uint2 *xt, uint2 *yt, float *amp, int32_t *src,
                            hipStream_t s)
{
    const int64_t n1 = (int64_t)M * Ppad;
    if (n1 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_freq_paths, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, paths, n,
                       Ppad, M, t_rep, pm);
    const int64_t n2 = (int64_t)M * (T + R) * Ppad;
    hipLaunchKernelGGL(k_freq_tables, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, pm, paths,
                       n, Ppad, M, tx, T, rx, R, f0c, dfc, xt, yt, amp, src);
    return hipGetLastError();
}

hipError_t launch_freq_gemm(const uint2 *xt, const uint2 *yt, const float *amp, const int32_t *src,
                            int T, int R, int M, int K, int64_t Ppad, int n_split, int64_t split_len,
                            float2 *partial, float2 *cube, hipStream_t s)
{
    if ((int64_t)n_split * split_len < Ppad || split_len % FQ_KS || Ppad % FQ_KS || Ppad <= 0)
        return hipErrorInvalidValue;
    FreqArgs A;
    A.xt = xt;
    A.yt = yt;
    A.amp = amp;
    A.src = src;
    A.T = T;
    A.R = R;
    A.M = M;
    A.K = K;
    A.Ppad = Ppad;
    A.tt = (T + FQ_TILE - 1) / FQ_TILE;
    A.rt = (R + FQ_TILE - 1) / FQ_TILE;
    A.n_split = n_split;
    A.split_len = split_len;
    A.partial = n_split > 1;
    A.out = n_split > 1 ? partial : cube;
    const int64_t blocks = (int64_t)n_split * M * A.tt * A.rt * K;
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_freq_gemm, dim3((unsigned)blocks), dim3(FQ_W * 64), 0, s, A);
    if (n_split > 1) {
        const int64_t per = (int64_t)M * K * T * R;
        hipLaunchKernelGGL(k_freq_reduce, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, s,
                           partial, n_split, T, R, M, K, cube);
    }
    return hipGetLastError();
}
