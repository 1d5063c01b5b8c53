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
// arithmetic.  A workgroup of four wavefronts computes a 96 x 96 (Tx x Rx)
// output tile of four consecutive samples of one chirp over one split of the
// paths, 16 paths per step, one sample per wavefront: the four share the
// step's table words (loaded once per workgroup, passed through LDS), and
// each wavefront generates its own X and Y fragments straight into operand
// registers and issues 108 v_mfma_f32_32x32x16_bf16 per step.  Operands are
// split bf16 hi + lo, products hi*hi + hi*lo + lo*hi, FP32 accumulation (as
// the separable GEMM).  Several path splits write partial tiles that a second
// kernel adds in split order (deterministic).
#include "rr_internal.h"

namespace {

#define FQ_G 4            // samples per workgroup, one per wavefront
#define FQ_KS 16          // paths per step
// a workgroup tile is NB x NB blocks of 32 x 32 (Tx x Rx), NB = 1, 2, 3; per
// step its table words are 8 NB chunks of 1 KiB (X and Y, NB blocks, 4 pieces)

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

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

// The paths of a synthesis: n records from `paths`, or, with rng_lo given,
// the records *rng_lo .. *rng_hi of `paths`, read on the device (a batched
// launch knows its scenes' path ranges only there), at most Ppad of them (the
// caller checks the count against its capacity afterwards).
struct PathRange {
    const SynPath *paths;
    int64_t n;
    const int64_t *rng_lo, *rng_hi;
};

// the path records and count of a synthesis, and the padded count the
// product reads (a multiple of FQ_KS; table entries beyond it are not needed)
__device__ __forceinline__ void path_range(const PathRange &R, int64_t Ppad, const SynPath *&p,
                                           int64_t &n, int64_t &used)
{
    if (R.rng_lo) {
        const int64_t lo = *R.rng_lo, hi = *R.rng_hi;
        p = R.paths + lo;
        n = min(max(hi - lo, (int64_t)0), Ppad);
        used = (n + FQ_KS - 1) / FQ_KS * FQ_KS;
    } else {
        p = R.paths;
        n = R.n;
        used = Ppad;
    }
}

// Per (chirp, path): first and last hit point at chirp time and the length
// between them.  Layout [M][Ppad] of 8 doubles: p1.xyz, pK.xyz, inner, amp.
__global__ void k_freq_paths(PathRange PR, int64_t Ppad, int M, double t_rep, double *pm)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const SynPath *paths;
    int64_t n, used;
    path_range(PR, Ppad, paths, n, used);
    if (g >= (int64_t)M * Ppad) return;
    const int m = (int)(g / Ppad);
    const int64_t p = g - (int64_t)m * Ppad;
    if (p >= used) return;
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
__global__ void k_freq_tables(const double *pm, PathRange PR, int64_t Ppad, int M, const double *tx,
                              int T, const double *rx, int R, double f0c, double dfc, uint2 *xt,
                              uint2 *yt, float *amp, int32_t *src)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const SynPath *paths;
    int64_t n, used;
    path_range(PR, Ppad, paths, n, used);
    const int64_t per_m = (int64_t)(T + R) * Ppad;
    if (g >= (int64_t)M * per_m) return;
    const int m = (int)(g / per_m);
    const int64_t rem = g - (int64_t)m * per_m;
    const int i = (int)(rem / Ppad);
    const int64_t p = rem - (int64_t)i * Ppad;
    if (p >= used) return;
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
    int kg;                   // groups of FQ_G samples
    int n_split;
    int64_t split_len;        // paths per split (multiple of FQ_KS)
    float2 *out;              // cube (one split) or partial tiles [split][m][k][T][R]
    int partial;
    // with rng_lo: the path count is *rng_hi - *rng_lo (at most Ppad), read
    // on the device, and the splits divide its padded count evenly
    const int64_t *rng_lo, *rng_hi;
};

// One workgroup: a 32 NB x 32 NB (Tx x Rx) tile of FQ_G consecutive samples
// of one chirp over one path split; wavefront w owns sample k0 + w and the
// whole tile (NB x NB blocks of 32 x 32, real and imaginary accumulators:
// 32 NB^2 registers).  The samples of a workgroup share the table words of
// every step: the (beta, gamma) words of the tile's Tx and Rx rows and 16
// paths, plus the paths' amplitudes and sources, are loaded once per
// workgroup (each lane fetching 2 NB 16-byte pieces a step ahead into
// registers) and passed through LDS (two buffers), already in the fragment
// lane order so that every read is a contiguous 1 KiB.  Each wavefront
// generates its own X and Y fragments for its sample.  Rows beyond the
// array's Tx and Rx counts read row 0's words and are never stored.
template <bool PER_EL, int NB>
__global__ __launch_bounds__(FQ_G * 64, NB == 3 || (NB == 2 && PER_EL) ? 1 : (NB == 2 ? 2 : 4)) void
k_freq_gemm(FreqArgs A)
{
    constexpr int CH = 8 * NB;            // table chunks per step
    constexpr int PL = CH / FQ_G;         // pieces per lane
    constexpr int TILE = 32 * NB;
    __shared__ uint4 Ls[2][CH + 1][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // the sample group fastest: the workgroups that share one split's tables
    // run together
    int64_t id = blockIdx.x;
    const int kq = (int)(id % A.kg);
    id /= A.kg;
    const int ri = (int)(id % A.rt);
    id /= A.rt;
    const int ti = (int)(id % A.tt);
    id /= A.tt;
    const int m = (int)(id % A.M);
    const int s = (int)(id / A.M);
    const int kw = kq * FQ_G + w;
    const bool kv = kw < A.K;
    const unsigned ku = (unsigned)(kv ? kw : A.K - 1);
    int64_t used = A.Ppad, split_len = A.split_len;
    if (A.rng_lo) {
        const int64_t n = min(max(*A.rng_hi - *A.rng_lo, (int64_t)0), A.Ppad);
        used = (n + FQ_KS - 1) / FQ_KS * FQ_KS;
        split_len = ((used + A.n_split - 1) / A.n_split + FQ_KS - 1) / FQ_KS * FQ_KS;
    }
    const int64_t pstart = (int64_t)s * split_len;
    const int64_t nsteps = max(min(used, pstart + split_len) - pstart, (int64_t)0) / FQ_KS;
    // an empty split still writes its (zero) tile; its loads stay at path 0
    const int64_t pbeg = nsteps > 0 ? pstart : 0;
    const int t0 = ti * TILE, r0 = ri * TILE;
    const int half = lane >> 5;

    // loader: this wavefront fetches chunks q = w + 4 j; chunk q is table
    // q / (4 NB) (X, Y), block (q % (4 NB)) / 4, piece q % 4 (paths 2 (q % 4)
    // and 2 (q % 4) + 1 of the lane's half); lane l reads row 32 block + l % 32
    const u32x4 *lp[PL];
#pragma unroll
    for (int j = 0; j < PL; j++) {
        const int q = w + FQ_G * j;
        const int tab = q / (4 * NB), blk = (q % (4 * NB)) >> 2, c = q & 3;
        int row = (tab ? r0 : t0) + 32 * blk + (lane & 31);
        if (row >= (tab ? A.R : A.T)) row = 0;    // any valid row: masked later
        const uint2 *base = tab ? A.yt + ((int64_t)m * A.R + row) * A.Ppad
                                : A.xt + ((int64_t)m * A.T + row) * A.Ppad;
        lp[j] = reinterpret_cast<const u32x4 *>(base + 8 * half + 2 * c);
    }
    // amplitudes and sources: wavefront 0, lanes 0-3 (amp) and 4-7 (src)
    const bool aload = w == 0 && lane < 8;
    const u32x4 *ap = lane < 4 ? reinterpret_cast<const u32x4 *>(A.amp) + (lane & 3)
                               : reinterpret_cast<const u32x4 *>(A.src) + (lane & 3);
    // one step's pieces of this lane, fetched a step ahead
    u32x4 P[PL], PA = {0u, 0u, 0u, 0u};
#define FQ_FETCH(p0)                                                                              \
    do {                                                                                          \
        const int64_t h_ = (p0) >> 1;                                                             \
        _Pragma("unroll") for (int j_ = 0; j_ < PL; j_++) P[j_] = lp[j_][h_];                     \
        if (aload) PA = ap[(p0) >> 2];                                                            \
    } while (0)
#define FQ_STASH(b_)                                                                              \
    do {                                                                                          \
        _Pragma("unroll") for (int j_ = 0; j_ < PL; j_++)                                         \
            *reinterpret_cast<u32x4 *>(&Ls[b_][w + FQ_G * j_][lane]) = P[j_];                     \
        if (aload) *reinterpret_cast<u32x4 *>(&Ls[b_][CH][lane]) = PA;                            \
    } while (0)
    auto raw_of = [&](int b, int q0) -> Raw {
        Raw r;
#pragma unroll
        for (int c = 0; c < 4; c++) r.w[c] = Ls[b][q0 + c][lane];
        return r;
    };

    f32x16 sr[NB][NB], si[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                sr[i][j][e] = 0.0f;
                si[i][j][e] = 0.0f;
            }

    FQ_FETCH(pbeg);
    FQ_STASH(0);
    FQ_FETCH(nsteps > 1 ? pbeg + FQ_KS : pbeg);
    __syncthreads();
    for (int64_t st = 0; st < nsteps; st++) {
        const int b = (int)(st & 1);
        // Y fragments of the Rx blocks (zero beyond the array)
        Frag y[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) y[j] = leg_frag(raw_of(b, 4 * NB + 4 * j), ku, nullptr);
        // amplitudes of the lane's 8 paths; in a per-element launch a path
        // feeds only its own transmitter's rows
        const uint4 a0 = Ls[b][CH][2 * half], a1 = Ls[b][CH][2 * half + 1];
        const uint4 s0 = Ls[b][CH][4 + 2 * half], s1 = Ls[b][CH][5 + 2 * half];
        const unsigned av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const unsigned sv[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const int t = t0 + 32 * i + (lane & 31);
            float a[8];
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int sp = (int)sv[e];
                a[e] = (!PER_EL || ((sp < 0) | (sp == t))) ? __uint_as_float(av[e]) : 0.0f;
            }
            const Frag x = leg_frag(raw_of(b, 4 * i), ku, a);
            const uint4 nih = neg(x.ih), nil = neg(x.il);
#pragma unroll
            for (int j = 0; j < NB; j++) {
                // re += Xr Yr - Xi Yi, im += Xr Yi + Xi Yr (hi*hi + hi*lo + lo*hi)
                sr[i][j] = MFMA(x.rh, y[j].rh, sr[i][j]);
                si[i][j] = MFMA(x.rh, y[j].ih, si[i][j]);
                sr[i][j] = MFMA(x.rh, y[j].rl, sr[i][j]);
                si[i][j] = MFMA(x.rh, y[j].il, si[i][j]);
                sr[i][j] = MFMA(x.rl, y[j].rh, sr[i][j]);
                si[i][j] = MFMA(x.rl, y[j].ih, si[i][j]);
                sr[i][j] = MFMA(nih, y[j].ih, sr[i][j]);
                si[i][j] = MFMA(x.ih, y[j].rh, si[i][j]);
                sr[i][j] = MFMA(nih, y[j].il, sr[i][j]);
                si[i][j] = MFMA(x.ih, y[j].rl, si[i][j]);
                sr[i][j] = MFMA(nil, y[j].ih, sr[i][j]);
                si[i][j] = MFMA(x.il, y[j].rh, si[i][j]);
            }
        }
        if (st + 1 < nsteps) FQ_STASH(b ^ 1);
        __syncthreads();
        FQ_FETCH(st + 2 < nsteps ? pbeg + (st + 2) * FQ_KS : pbeg);
    }
#undef FQ_FETCH
#undef FQ_STASH
    // D layout: register e of lane l is row 8 (e / 4) + 4 (l / 32) + e % 4
    // (a Tx row of block i), column l % 32 (an Rx column of block j)
    if (!kv) return;
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int to = t0 + 32 * i + 8 * (e >> 2) + 4 * half + (e & 3);
                const int ro = r0 + 32 * j + (lane & 31);
                if (to < A.T && ro < A.R) {
                    const float2 v = make_float2(sr[i][j][e], si[i][j][e]);
                    if (A.partial)
                        A.out[((((int64_t)s * A.M + m) * A.K + kw) * A.T + to) * A.R + ro] = v;
                    else
                        A.out[(((int64_t)to * A.R + ro) * A.M + m) * A.K + kw] = v;
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
int freq_k_group() { return FQ_G; }

hipError_t launch_freq_prep(const SynPath *paths, int64_t n, const int64_t *rng_lo,
                            const int64_t *rng_hi, int64_t Ppad, int M, double t_rep,
                            const double *tx, int T, const double *rx, int R, double f0c, double dfc,
                            double *pm, uint2 *xt, uint2 *yt, float *amp, int32_t *src,
                            hipStream_t s)
{
    const int64_t n1 = (int64_t)M * Ppad;
    if (n1 <= 0) return hipSuccess;
    PathRange PR{paths, n, rng_lo, rng_hi};
    hipLaunchKernelGGL(k_freq_paths, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, PR, Ppad,
                       M, t_rep, pm);
    const int64_t n2 = (int64_t)M * (T + R) * Ppad;
    hipLaunchKernelGGL(k_freq_tables, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, pm, PR,
                       Ppad, M, tx, T, rx, R, f0c, dfc, xt, yt, amp, src);
    return hipGetLastError();
}

// workgroup tile of NB blocks of 32 (1, 2 or 3) that wastes the least
// padding on a T x R array (ties: the larger tile)
int freq_tile_blocks(int T, int R)
{
    int best = 3;
    int64_t best_area = -1;
    for (int nb = 3; nb >= 1; nb--) {
        const int64_t t = 32 * nb, area = ((T + t - 1) / t * t) * ((R + t - 1) / t * t);
        if (best_area < 0 || area < best_area) {
            best_area = area;
            best = nb;
        }
    }
    return best;
}

hipError_t launch_freq_gemm(const uint2 *xt, const uint2 *yt, const float *amp, const int32_t *src,
                            int T, int R, int M, int K, int64_t Ppad, int n_split, int64_t split_len,
                            int per_element, int nb, const int64_t *rng_lo, const int64_t *rng_hi,
                            float2 *partial, float2 *cube, hipStream_t s)
{
    if ((int64_t)n_split * split_len < Ppad || split_len % FQ_KS || Ppad % FQ_KS || Ppad <= 0)
        return hipErrorInvalidValue;
    if (nb < 1 || nb > 3) return hipErrorInvalidValue;
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
    A.tt = (T + 32 * nb - 1) / (32 * nb);
    A.rt = (R + 32 * nb - 1) / (32 * nb);
    A.kg = (K + FQ_G - 1) / FQ_G;
    A.n_split = n_split;
    A.split_len = split_len;
    A.partial = n_split > 1;
    A.out = n_split > 1 ? partial : cube;
    A.rng_lo = rng_lo;
    A.rng_hi = rng_hi;
    const int64_t blocks = (int64_t)n_split * M * A.tt * A.rt * A.kg;
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const dim3 g((unsigned)blocks), t(FQ_G * 64);
    switch (nb * 2 + (per_element ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((k_freq_gemm<false, 1>), g, t, 0, s, A); break;
    case 3: hipLaunchKernelGGL((k_freq_gemm<true, 1>), g, t, 0, s, A); break;
    case 4: hipLaunchKernelGGL((k_freq_gemm<false, 2>), g, t, 0, s, A); break;
    case 5: hipLaunchKernelGGL((k_freq_gemm<true, 2>), g, t, 0, s, A); break;
    case 6: hipLaunchKernelGGL((k_freq_gemm<false, 3>), g, t, 0, s, A); break;
    default: hipLaunchKernelGGL((k_freq_gemm<true, 3>), g, t, 0, s, A); break;
    }
    if (n_split > 1) {
        const int64_t per = (int64_t)M * K * T * R;
        hipLaunchKernelGGL(k_freq_reduce, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, s,
                           partial, n_split, T, R, M, K, cube);
    }
    return hipGetLastError();
}
