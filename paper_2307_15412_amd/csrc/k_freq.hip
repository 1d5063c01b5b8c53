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
// arithmetic.  A workgroup of four wavefronts computes a square (Tx x Rx)
// output tile of four consecutive samples of one chirp over one split of the
// paths, one sample per wavefront: the four share the step's table words
// (loaded once per workgroup, passed through LDS), and each wavefront
// generates its own X and Y fragments straight into operand registers.  The
// tile is 16 or 48 wide in 16 x 16 blocks (v_mfma_f32_16x16x32_bf16, 32 paths
// a step) or 32, 64 or 96 wide in 32 x 32 blocks (v_mfma_f32_32x32x16_bf16,
// 16 paths a step), chosen per array to trade padding against the sharing of
// phasors among products.  Operands are split bf16 hi + lo, products
// hi*hi + hi*lo + lo*hi, FP32 accumulation (as the separable GEMM).  Several
// path splits write partial tiles that a second kernel adds in split order
// (deterministic).
#include "rr_internal.h"

namespace {

#define FQ_G 4            // samples per workgroup, one per wavefront
#define FQ_PAD 32         // path granule of the tables and splits (a multiple of every step)
#define FQ_KS_KMAX 1024   // most samples of the sample split (2 x 2 blocks of 16 x 16 = 32 x 32)
// a workgroup tile is NB x NB blocks of 32 x 32 (Tx x Rx), NB = 1, 2, 3; per
// step its table words are 8 NB chunks of 1 KiB (X and Y, NB blocks, 4 pieces)

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double frac(double x) { return x - floor(x); }

// frac(x) as 32-bit fixed-point turns, rounded to nearest (2^32 wraps to 0)
__device__ __forceinline__ unsigned turns_u32(double x)
{
    const double r = rint(frac(x) * 4294967296.0);
    return r >= 4294967296.0 ? 0u : (unsigned)r;
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
// product reads (a multiple of FQ_PAD; table entries beyond it are not needed)
__device__ __forceinline__ void path_range(const PathRange &R, int64_t Ppad, const SynPath *&p,
                                           int64_t &n, int64_t &used)
{
    if (R.rng_lo) {
        const int64_t lo = *R.rng_lo, hi = *R.rng_hi;
        p = R.paths + lo;
        n = min(max(hi - lo, (int64_t)0), Ppad);
        used = (n + FQ_PAD - 1) / FQ_PAD * FQ_PAD;
    } else {
        p = R.paths;
        n = R.n;
        used = Ppad;
    }
}

// Leg tables, one thread per path over a share of the chirps: the first and
// last hit point at chirp time and the length between them, then per element
// the leg in fixed-point turns (beta, gamma): xt[m][t][p] of
// dX = |p1 - tx_t| + inner and yt[m][r][p] of dY = |rx_r - pK|; and per path
// the amplitude (0 beyond the path count) and source.  OWN_TX (per-element
// launch, sample split): the channels of transmitter t read only the paths of
// t's group, so only each path's own transmitter word is kept, xt[m][0][p].
template <bool OWN_TX>
__global__ __launch_bounds__(256) void k_freq_legs(PathRange PR, int64_t Ppad, int M, double t_rep,
                                                   const double *tx, int T, const double *rx,
                                                   int R, double f0c, double dfc, uint2 *xt,
                                                   uint2 *yt, float *amp, int32_t *src)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const SynPath *paths;
    int64_t n, used;
    path_range(PR, Ppad, paths, n, used);
    if (p >= used) return;
    const int XR = OWN_TX ? 1 : T;
    if (p >= n) {
        for (int m = blockIdx.y; m < M; m += gridDim.y) {
            for (int i = 0; i < XR; i++) xt[((int64_t)m * XR + i) * Ppad + p] = make_uint2(0u, 0u);
            for (int i = 0; i < R; i++) yt[((int64_t)m * R + i) * Ppad + p] = make_uint2(0u, 0u);
        }
        if (blockIdx.y == 0) {
            amp[p] = 0.0f;
            src[p] = -1;
        }
        return;
    }
    const SynPath &P = paths[p];
    const int K = P.K;
    const int t_own = OWN_TX ? min(max(P.src, 0), T - 1) : 0;
    double h[RR_KMAX][3], v[RR_KMAX][3];   // the path's points, held over the chirps
#pragma unroll
    for (int j = 0; j < RR_KMAX; j++)
#pragma unroll
        for (int a = 0; a < 3; a++) {
            h[j][a] = j < K ? P.P[j][a] : 0.0;
            v[j][a] = j < K ? P.V[j][a] : 0.0;
        }
    for (int m = blockIdx.y; m < M; m += gridDim.y) {
        const double tau = (double)m * t_rep;
        double q1[3], qk[3], inner = 0.0;
        for (int a = 0; a < 3; a++) q1[a] = h[0][a] + v[0][a] * tau;
        for (int a = 0; a < 3; a++) qk[a] = q1[a];
#pragma unroll
        for (int j = 1; j < RR_KMAX; j++) {
            if (j >= K) break;
            double q[3];
            for (int a = 0; a < 3; a++) q[a] = h[j][a] + v[j][a] * tau;
            inner += dist3(q, qk);
            for (int a = 0; a < 3; a++) qk[a] = q[a];
        }
        uint2 *xo = xt + (int64_t)m * XR * Ppad + p;
        for (int i = 0; i < XR; i++) {
            const double d = dist3(q1, tx + 3 * (OWN_TX ? t_own : i)) + inner;
            xo[(int64_t)i * Ppad] = make_uint2(turns_u32(d * f0c), turns_u32(d * dfc));
        }
        uint2 *yo = yt + (int64_t)m * R * Ppad + p;
        for (int i = 0; i < R; i++) {
            const double d = dist3(rx + 3 * i, qk);
            yo[(int64_t)i * Ppad] = make_uint2(turns_u32(d * f0c), turns_u32(d * dfc));
        }
    }
    if (blockIdx.y == 0) {
        amp[p] = (float)P.amp;
        src[p] = P.src;
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

typedef float f32x4 __attribute__((ext_vector_type(4)));

// one split-bf16 product on the matrix cores: 32 x 32 blocks of 16 paths, or
// 16 x 16 blocks of 32 paths
template <int BS> struct Mfma;
template <> struct Mfma<32> {
    typedef f32x16 acc;
    static __device__ __forceinline__ acc mma(uint4 a, uint4 b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf(a), as_bf(b), c, 0, 0, 0);
    }
};
template <> struct Mfma<16> {
    typedef f32x4 acc;
    static __device__ __forceinline__ acc mma(uint4 a, uint4 b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a), as_bf(b), c, 0, 0, 0);
    }
};

// exp(-j 2 pi u) of fixed-point turns u: the top 23 bits of u become the
// mantissa of a float in [1, 2) turns (one funnel shift), which the hardware
// sine and cosine (arguments in turns) take as they are; the phase keeps
// 2^-23 turns (7.5e-7 rad)
__device__ __forceinline__ void phasor(unsigned u, float &re, float &im)
{
    const float f = __uint_as_float(__builtin_amdgcn_alignbit(0x7fu, u, 9u));
    re = __builtin_amdgcn_cosf(f);
    im = -__builtin_amdgcn_sinf(f);
}

struct Frag {          // one operand fragment (8 values a lane), split: real hi/lo, imaginary hi/lo
    uint4 rh, rl, ih, il;
};

struct Raw {           // one lane's table words of one step: 8 (beta, gamma) pairs
    uint4 w[4];
};

// the 8 path slots of one fragment lane at sample k, times a (when given),
// split into the four bf16 planes
// hi = bf16(x, y); lo = bf16(x - hi.x, y - hi.y) with each difference formed
// exactly by one dot product, hi . (-1, -0) + x and hi . (0, -1) + y: one
// vector instruction instead of a shift or mask and a subtraction.  Used
// where the matrix cores are mostly idle (the sample split): the dot products
// do not overlap the MFMAs, which costs the Tx x Rx tiles more than it saves.
// The (-1, -0) word must be a literal: as the inline constant -1.0 the
// hardware reads it as the 32-bit float, i.e. (0, -1).
__device__ __forceinline__ void split_bf16_dot(float x, float y, unsigned &hi, unsigned &lo)
{
    hi = pack_bf16(x, y);
    const bf16x2 h = __builtin_bit_cast(bf16x2, hi);
    lo = pack_bf16(__builtin_amdgcn_fdot2_f32_bf16(h, __builtin_bit_cast(bf16x2, 0x8000bf80u), x, false),
                   __builtin_amdgcn_fdot2_f32_bf16(h, __builtin_bit_cast(bf16x2, 0xbf800000u), y, false));
}

// one operand fragment from the lane's 8 phases (32-bit fixed-point turns):
// the phasors, times the amplitudes a (if given), split into bf16 hi/lo
__device__ __forceinline__ Frag phase_frag(const unsigned *ph, const float *a)
{
    float re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
        phasor(ph[e], re[e], im[e]);
        if (a) {
            re[e] *= a[e];
            im[e] *= a[e];
        }
    }
    Frag f;
    unsigned *rh = &f.rh.x, *rl = &f.rl.x, *ih = &f.ih.x, *il = &f.il.x;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        split_bf16_dot(re[2 * q], re[2 * q + 1], rh[q], rl[q]);
        split_bf16_dot(im[2 * q], im[2 * q + 1], ih[q], il[q]);
    }
    return f;
}

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
    int64_t split_len;        // paths per split (multiple of FQ_PAD)
    float2 *out;              // cube (one split) or partial tiles [split][m][k][T][R]
    int partial;
    // with rng_lo: the path count is *rng_hi - *rng_lo (at most Ppad), read
    // on the device, and the splits divide its padded count evenly
    const int64_t *rng_lo, *rng_hi;
    // sample split (one channel per wavefront): k = k1 S + k2, S = 2^S_log2
    int S, S_log2;
    int64_t n_waves;
    // per-element launch, sample split: groups[t] .. groups[t + 1] are the
    // paths of transmitter t (path indices of the list the tables were built
    // from, plus groups[0]); a channel's wavefronts read only those
    const int64_t *groups;
};

// One workgroup: a BS NB x BS NB (Tx x Rx) tile of FQ_G consecutive samples
// of one chirp over one path split, in NB x NB blocks of BS x BS (BS = 32:
// v_mfma_f32_32x32x16_bf16, 16 paths a step; BS = 16:
// v_mfma_f32_16x16x32_bf16, 32 paths a step).  Wavefront w owns sample
// k0 + w and the whole tile (real and imaginary accumulators: 2 NB^2 BS^2 / 64
// registers).  The samples of a workgroup share the table words of every
// step: the (beta, gamma) words of the tile's Tx and Rx rows and the step's
// paths, plus the paths' amplitudes and sources, are loaded once per
// workgroup (each lane fetching 2 NB 16-byte pieces a step ahead into
// registers) and passed through LDS (two buffers), already in the fragment
// lane order so that every read is a contiguous 1 KiB.  Each wavefront
// generates its own X and Y fragments for its sample.  Rows beyond the
// array's Tx and Rx counts read row 0's words and are never stored.
template <bool PER_EL, int BS, int NB>
__global__ __launch_bounds__(FQ_G * 64, BS == 16 ? (NB == 1 ? 4 : 2)
                                                 : (NB == 3 || (NB == 2 && PER_EL) ? 1 : (NB == 2 ? 2 : 4)))
void k_freq_gemm(FreqArgs A)
{
    typedef typename Mfma<BS>::acc acc;
    constexpr int GR = 64 / BS;           // lane groups: each holds 8 paths of a fragment row
    constexpr int STEP = 8 * GR;          // paths per step
    constexpr int NE = BS * BS / 64;      // accumulator registers of a block
    constexpr int CH = 8 * NB;            // 1 KiB table chunks per step (X and Y, NB blocks, 4 pieces)
    constexpr int PL = CH / FQ_G;         // pieces per lane
    constexpr int TILE = BS * NB;
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
        used = (n + FQ_PAD - 1) / FQ_PAD * FQ_PAD;
        split_len = ((used + A.n_split - 1) / A.n_split + FQ_PAD - 1) / FQ_PAD * FQ_PAD;
    }
    const int64_t pstart = (int64_t)s * split_len;
    const int64_t nsteps = max(min(used, pstart + split_len) - pstart, (int64_t)0) / STEP;
    // an empty split still writes its (zero) tile; its loads stay at path 0
    const int64_t pbeg = nsteps > 0 ? pstart : 0;
    const int t0 = ti * TILE, r0 = ri * TILE;
    const int grp = lane / BS, lrow = lane % BS;

    // loader: this wavefront fetches chunks q = w + 4 j; chunk q is table
    // q / (4 NB) (X, Y), block (q % (4 NB)) / 4, piece q % 4 (paths 2 (q % 4)
    // and 2 (q % 4) + 1 of the lane group's 8); lane l reads row
    // BS block + l % BS
    const u32x4 *lp[PL];
#pragma unroll
    for (int j = 0; j < PL; j++) {
        const int q = w + FQ_G * j;
        const int tab = q / (4 * NB), blk = (q % (4 * NB)) >> 2, c = q & 3;
        int row = (tab ? r0 : t0) + BS * blk + lrow;
        if (row >= (tab ? A.R : A.T)) row = 0;    // any valid row: masked later
        const uint2 *base = tab ? A.yt + ((int64_t)m * A.R + row) * A.Ppad
                                : A.xt + ((int64_t)m * A.T + row) * A.Ppad;
        lp[j] = reinterpret_cast<const u32x4 *>(base + 8 * grp + 2 * c);
    }
    // amplitudes and sources of a step: wavefront 0, lanes 0 .. STEP/4 - 1
    // (amp) and STEP/4 .. STEP/2 - 1 (src)
    const bool aload = w == 0 && lane < STEP / 2;
    const u32x4 *ap = lane < STEP / 4 ? reinterpret_cast<const u32x4 *>(A.amp) + lane
                                      : reinterpret_cast<const u32x4 *>(A.src) + (lane - STEP / 4);
    // one step's pieces of this lane, fetched a step ahead (native vector
    // registers: an array of HIP's uint4 would be kept in scratch memory)
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

    acc sr[NB][NB], si[NB][NB];
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
            for (int e = 0; e < NE; e++) {
                sr[i][j][e] = 0.0f;
                si[i][j][e] = 0.0f;
            }

    FQ_FETCH(pbeg);
    FQ_STASH(0);
    FQ_FETCH(nsteps > 1 ? pbeg + STEP : pbeg);
    __syncthreads();
    for (int64_t st = 0; st < nsteps; st++) {
        const int b = (int)(st & 1);
        // Y fragments of the Rx blocks (zero beyond the array)
        Frag y[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) y[j] = leg_frag(raw_of(b, 4 * NB + 4 * j), ku, nullptr);
        // amplitudes of the lane's 8 paths; in a per-element launch a path
        // feeds only its own transmitter's rows
        const uint4 a0 = Ls[b][CH][2 * grp], a1 = Ls[b][CH][2 * grp + 1];
        const uint4 s0 = Ls[b][CH][STEP / 4 + 2 * grp], s1 = Ls[b][CH][STEP / 4 + 2 * grp + 1];
        const unsigned av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const unsigned sv[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const int t = t0 + BS * i + lrow;
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
                sr[i][j] = Mfma<BS>::mma(x.rh, y[j].rh, sr[i][j]);
                si[i][j] = Mfma<BS>::mma(x.rh, y[j].ih, si[i][j]);
                sr[i][j] = Mfma<BS>::mma(x.rh, y[j].rl, sr[i][j]);
                si[i][j] = Mfma<BS>::mma(x.rh, y[j].il, si[i][j]);
                sr[i][j] = Mfma<BS>::mma(x.rl, y[j].rh, sr[i][j]);
                si[i][j] = Mfma<BS>::mma(x.rl, y[j].ih, si[i][j]);
                sr[i][j] = Mfma<BS>::mma(nih, y[j].ih, sr[i][j]);
                si[i][j] = Mfma<BS>::mma(x.ih, y[j].rh, si[i][j]);
                sr[i][j] = Mfma<BS>::mma(nih, y[j].il, sr[i][j]);
                si[i][j] = Mfma<BS>::mma(x.ih, y[j].rl, si[i][j]);
                sr[i][j] = Mfma<BS>::mma(nil, y[j].ih, sr[i][j]);
                si[i][j] = Mfma<BS>::mma(x.il, y[j].rh, si[i][j]);
            }
        }
        if (st + 1 < nsteps) FQ_STASH(b ^ 1);
        __syncthreads();
        FQ_FETCH(st + 2 < nsteps ? pbeg + (st + 2) * STEP : pbeg);
    }
#undef FQ_FETCH
#undef FQ_STASH
    // D layout: register e of lane l is row 8 (e / 4) + 4 (l / 32) + e % 4
    // (BS = 32) or 4 (l / 16) + e (BS = 16) of the block, column l % BS
    if (!kv) return;
#pragma unroll
    for (int i = 0; i < NB; i++)
#pragma unroll
        for (int j = 0; j < NB; j++)
#pragma unroll
            for (int e = 0; e < NE; e++) {
                const int br = BS == 32 ? 8 * (e >> 2) + 4 * grp + (e & 3) : 4 * grp + e;
                const int to = t0 + BS * i + br;
                const int ro = r0 + BS * j + lrow;
                if (to < A.T && ro < A.R) {
                    const float2 v = make_float2(sr[i][j][e], si[i][j][e]);
                    if (A.partial)
                        A.out[((((int64_t)s * A.M + m) * A.K + kw) * A.T + to) * A.R + ro] = v;
                    else
                        A.out[(((int64_t)to * A.R + ro) * A.M + m) * A.K + kw] = v;
                }
            }
}

// One wavefront per (path split, chirp, channel): the channel's samples as a
// product over paths.  With beta and gamma of channel (t, r) the sums of its
// Tx and Rx leg words, the phase of sample k = k1 S + k2 splits exactly (in
// 32-bit fixed-point turns) as (beta + k1 S gamma) + k2 gamma, so
//     s[k1 S + k2] = sum_p U[k1, p] V[p, k2],
//     U[k1, p] = a_p exp(-j 2 pi (beta + k1 S gamma)),  V[p, k2] = exp(-j 2 pi k2 gamma),
// a (Q x paths) by (paths x S) complex product in QB x SB blocks of 16 x 16
// (v_mfma_f32_16x16x32_bf16, 32 paths a step, split bf16 as the tile
// kernels, the low parts by one dot product each).  Per path and channel it evaluates Q + S phasors instead of the
// Tx x Rx tiles' (T + R) K / (T R): the better choice for small arrays.  Each
// lane loads its 8 paths' leg words straight from the tables (the 16 lanes of
// a row group read the same words).
// the shared-launch 1 x 1 variant fits three wavefronts per SIMD without
// spilling (3-7 % faster than two); the others spill at three and run two
// (asked for explicitly: left to itself the compiler parks registers in the
// accumulator file and moves them back and forth every step)
template <bool PER_EL, int QB, int SB>
__global__ __launch_bounds__(FQ_G * 64, (!PER_EL && QB * SB == 1) ? 3 : 2) void k_freq_ks(FreqArgs A)
{
    typedef f32x4 acc;
    const int lane = threadIdx.x & 63;
    // wavefront index, uniform by construction (kept in scalar registers)
    const int64_t wv = (int64_t)blockIdx.x * FQ_G + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wv >= A.n_waves) return;
    // wave -> (split, chirp, channel), channel fastest
    const int C = A.T * A.R;
    int64_t id = wv;
    const int c = (int)(id % C);
    id /= C;
    const int m = (int)(id % A.M);
    const int s = (int)(id / A.M);
    const int t = c / A.R, r = c - t * A.R;
    int64_t used = A.Ppad, split_len = A.split_len;
    if (A.rng_lo) {
        const int64_t n = min(max(*A.rng_hi - *A.rng_lo, (int64_t)0), A.Ppad);
        used = (n + FQ_PAD - 1) / FQ_PAD * FQ_PAD;
        split_len = ((used + A.n_split - 1) / A.n_split + FQ_PAD - 1) / FQ_PAD * FQ_PAD;
    }
    // the paths this channel reads: all, or (per-element) its transmitter's
    // group widened to whole 32-path steps (the paths of neighbouring groups
    // in the edge steps are masked by their source below)
    int64_t plo = 0, phi = used;
    // [glo, ghi): the group itself; steps inside it hold only paths of this
    // transmitter and need no masking
    int64_t glo = 0, ghi = -1;
    if (PER_EL && A.groups) {
        const int64_t g0 = A.groups[0];
        glo = min(max(A.groups[t] - g0, (int64_t)0), used);
        ghi = min(max(A.groups[t + 1] - g0, (int64_t)0), used);
        plo = glo / 32 * 32;
        phi = min((ghi + 31) / 32 * 32, used);
        phi = max(phi, plo);
        split_len = ((phi - plo + A.n_split - 1) / A.n_split + 31) / 32 * 32;
    }
    const int64_t pstart = plo + (int64_t)s * split_len;
    const int64_t nsteps = max(min(phi, pstart + split_len) - pstart, (int64_t)0) / 32;
    const int grp = lane >> 4, lrow = lane & 15;
    // the lane's 8 paths of a step: pstart + 32 step + 8 grp + (0 .. 7)
    const int64_t p0 = nsteps > 0 ? pstart + 8 * grp : 0;
    // X words: per-element launches with groups keep one row per chirp (each
    // path's own transmitter), otherwise one per (chirp, transmitter)
    const int64_t xrow = PER_EL && A.groups ? (int64_t)m : (int64_t)m * A.T + t;
    const u32x4 *xp = reinterpret_cast<const u32x4 *>(A.xt + xrow * A.Ppad + p0);
    const u32x4 *yp = reinterpret_cast<const u32x4 *>(A.yt + ((int64_t)m * A.R + r) * A.Ppad + p0);
    const u32x4 *apn = reinterpret_cast<const u32x4 *>(A.amp + p0);
    const u32x4 *spn = reinterpret_cast<const u32x4 *>(A.src + p0);
    // sample k1 S + k2 of the lane's U row k1 = 16 q + lrow and V column
    // k2 = 16 b + lrow: with t = lrow gamma (mod 2^32) the V phase is
    // t + 16 b gamma and the U phase beta + ((t + 16 q gamma) << S_log2)
    const unsigned lr = (unsigned)lrow;
    const int ssh = A.S_log2;
    f32x4 sr[QB][SB], si[QB][SB];
#pragma unroll
    for (int i = 0; i < QB; i++)
#pragma unroll
        for (int j = 0; j < SB; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                sr[i][j][e] = 0.0f;
                si[i][j][e] = 0.0f;
            }
    // a step's words, loaded a step ahead into the other of two register
    // sets (the loop is unrolled by two, so no copies between the sets)
    u32x4 X0[4], Y0[4], AM0[2], SR0[2], X1[4], Y1[4], AM1[2], SR1[2];
#define KS_LOAD(st_, X, Y, AM, SR)                                                                \
    do {                                                                                          \
        const int64_t o_ = (st_) * 16;                                                            \
        _Pragma("unroll") for (int q_ = 0; q_ < 4; q_++) {                                        \
            X[q_] = xp[o_ + q_];                                                                  \
            Y[q_] = yp[o_ + q_];                                                                  \
        }                                                                                         \
        AM[0] = apn[(st_) * 8];                                                                   \
        AM[1] = apn[(st_) * 8 + 1];                                                               \
        if (PER_EL) {                                                                             \
            SR[0] = spn[(st_) * 8];                                                               \
            SR[1] = spn[(st_) * 8 + 1];                                                           \
        }                                                                                         \
    } while (0)
    // one step: the channel's (beta, gamma) per path (sums of its Tx and Rx
    // leg words), the U and V phases from one product t = lrow gamma, the
    // amplitudes (in a per-element launch a path feeds its own Tx only: other
    // transmitters' paths, present only in a group's edge steps, get 0), the
    // fragments and the products
#define KS_STEP(X, Y, AM, SR, ST)                                                                 \
    do {                                                                                          \
        unsigned bt_[8], gm_[8], t_[8], ph_[8];                                                   \
        float a_[8];                                                                              \
        _Pragma("unroll") for (int q_ = 0; q_ < 4; q_++) {                                        \
            bt_[2 * q_] = X[q_].x + Y[q_].x;                                                      \
            gm_[2 * q_] = X[q_].y + Y[q_].y;                                                      \
            bt_[2 * q_ + 1] = X[q_].z + Y[q_].z;                                                  \
            gm_[2 * q_ + 1] = X[q_].w + Y[q_].w;                                                  \
        }                                                                                         \
        _Pragma("unroll") for (int e_ = 0; e_ < 8; e_++) t_[e_] = lr * gm_[e_];                   \
        _Pragma("unroll") for (int e_ = 0; e_ < 4; e_++) {                                        \
            a_[e_] = __uint_as_float(AM[0][e_]);                                                  \
            a_[4 + e_] = __uint_as_float(AM[1][e_]);                                              \
        }                                                                                         \
        if (PER_EL) {                                                                             \
            const int64_t ps_ = pstart + 32 * (int64_t)(ST);                                      \
            if (ghi < 0 || ps_ < glo || ps_ + 32 > ghi) {                                         \
                _Pragma("unroll") for (int e_ = 0; e_ < 4; e_++) {                                \
                    const int s0_ = (int)SR[0][e_], s1_ = (int)SR[1][e_];                         \
                    if (s0_ >= 0 && s0_ != t) a_[e_] = 0.0f;                                      \
                    if (s1_ >= 0 && s1_ != t) a_[4 + e_] = 0.0f;                                  \
                }                                                                                 \
            }                                                                                     \
        }                                                                                         \
        Frag v_[SB];                                                                              \
        _Pragma("unroll") for (int j_ = 0; j_ < SB; j_++) {                                       \
            _Pragma("unroll") for (int e_ = 0; e_ < 8; e_++)                                      \
                ph_[e_] = j_ ? t_[e_] + (unsigned)j_ * (gm_[e_] << 4) : t_[e_];                   \
            v_[j_] = phase_frag(ph_, nullptr);                                                    \
        }                                                                                         \
        _Pragma("unroll") for (int i_ = 0; i_ < QB; i_++) {                                       \
            _Pragma("unroll") for (int e_ = 0; e_ < 8; e_++)                                      \
                ph_[e_] = bt_[e_] + ((i_ ? t_[e_] + (unsigned)i_ * (gm_[e_] << 4) : t_[e_]) << ssh); \
            const Frag x_ = phase_frag(ph_, a_);                                                  \
            const uint4 nih_ = neg(x_.ih), nil_ = neg(x_.il);                                     \
            _Pragma("unroll") for (int j_ = 0; j_ < SB; j_++) {                                   \
                acc &R_ = sr[i_][j_], &I_ = si[i_][j_];                                           \
                R_ = Mfma<16>::mma(x_.rh, v_[j_].rh, R_);                                         \
                I_ = Mfma<16>::mma(x_.rh, v_[j_].ih, I_);                                         \
                R_ = Mfma<16>::mma(x_.rh, v_[j_].rl, R_);                                         \
                I_ = Mfma<16>::mma(x_.rh, v_[j_].il, I_);                                         \
                R_ = Mfma<16>::mma(x_.rl, v_[j_].rh, R_);                                         \
                I_ = Mfma<16>::mma(x_.rl, v_[j_].ih, I_);                                         \
                R_ = Mfma<16>::mma(nih_, v_[j_].ih, R_);                                          \
                I_ = Mfma<16>::mma(x_.ih, v_[j_].rh, I_);                                         \
                R_ = Mfma<16>::mma(nih_, v_[j_].il, R_);                                          \
                I_ = Mfma<16>::mma(x_.ih, v_[j_].rl, I_);                                         \
                R_ = Mfma<16>::mma(nil_, v_[j_].ih, R_);                                          \
                I_ = Mfma<16>::mma(x_.il, v_[j_].rh, I_);                                         \
            }                                                                                     \
        }                                                                                         \
    } while (0)
    if (nsteps > 0) KS_LOAD(0, X0, Y0, AM0, SR0);
    for (int64_t st = 0; st < nsteps; st += 2) {
        if (st + 1 < nsteps) KS_LOAD(st + 1, X1, Y1, AM1, SR1);
        KS_STEP(X0, Y0, AM0, SR0, st);
        if (st + 1 >= nsteps) break;
        if (st + 2 < nsteps) KS_LOAD(st + 2, X0, Y0, AM0, SR0);
        KS_STEP(X1, Y1, AM1, SR1, st + 1);
    }
#undef KS_LOAD
#undef KS_STEP
    // D layout: register e of lane l is row 4 (l / 16) + e (k1), column
    // l % 16 (k2) of the block
#pragma unroll
    for (int i = 0; i < QB; i++)
#pragma unroll
        for (int j = 0; j < SB; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int kk1 = 16 * i + 4 * grp + e, kk2 = 16 * j + lrow;
                const int k = kk1 * A.S + kk2;
                if (kk2 >= A.S || k >= A.K) continue;
                const float2 v = make_float2(sr[i][j][e], si[i][j][e]);
                if (A.partial)
                    A.out[((((int64_t)s * A.M + m) * A.K + k) * A.T + t) * A.R + r] = v;
                else
                    A.out[((int64_t)c * A.M + m) * A.K + k] = v;
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

int freq_k_step() { return FQ_PAD; }
int freq_k_group() { return FQ_G; }

hipError_t launch_freq_prep(const SynPath *paths, int64_t n, const int64_t *rng_lo,
                            const int64_t *rng_hi, int64_t Ppad, int M, double t_rep,
                            const double *tx, int T, bool own_tx, const double *rx, int R,
                            double f0c, double dfc, uint2 *xt, uint2 *yt, float *amp, int32_t *src,
                            hipStream_t s)
{
    if (M <= 0 || Ppad <= 0) return hipSuccess;
    PathRange PR{paths, n, rng_lo, rng_hi};
    // one thread per path; the chirps shared over enough workgroups to fill
    // the chip (each thread keeps its path's points over its chirps)
    const int64_t bx = (Ppad + 255) / 256;
    const int by = (int)std::min<int64_t>(M, std::max<int64_t>(1, (4096 + bx - 1) / bx));
    const dim3 g((unsigned)bx, (unsigned)by);
    if (own_tx)
        hipLaunchKernelGGL(k_freq_legs<true>, g, dim3(256), 0, s, PR, Ppad, M, t_rep, tx, T, rx, R,
                           f0c, dfc, xt, yt, amp, src);
    else
        hipLaunchKernelGGL(k_freq_legs<false>, g, dim3(256), 0, s, PR, Ppad, M, t_rep, tx, T, rx, R,
                           f0c, dfc, xt, yt, amp, src);
    return hipGetLastError();
}

// workgroup tile of NB blocks of 32 (1, 2 or 3) that wastes the least
// padding on a T x R array (ties: the larger tile)
// Product layouts: Tx x Rx tiles (square; 16 and 48 in 16 x 16 blocks, 32,
// 64 and 96 in 32 x 32 blocks), or tile 1: one channel per wavefront with the
// samples split (k = k1 S + k2).  Measured throughput per padded output
// (split-bf16 products, 1e12 complex multiply-adds/s on one MI355X): bigger
// tiles share each phasor among more products; the 16 x 16 blocks cost more
// per output than 32 x 32 at equal tile; the sample split pads nothing across
// channels and shares each phasor among ~sqrt(K) samples.  The layout that
// minimises padded outputs / throughput.
static const int FQ_TILES[5] = {16, 32, 48, 64, 96};
static const double FQ_TILE_RATE[5] = {17.8, 30.0, 38.0, 43.0, 42.0};

// sample split of K samples: QB x SB blocks of 16 x 16, S samples a row
// blocks of the sample split and S = 2^s, the least power of two with
// Q S >= K (Q = 16 qb rows); S <= 16 sb always holds
static void ks_shape(int K, int &qb, int &sb, int &S, int &s)
{
    qb = K <= 512 ? 1 : 2;
    sb = K <= 256 ? 1 : 2;
    const int need = (K + 16 * qb - 1) / (16 * qb);
    s = 0;
    while ((1 << s) < need) s++;
    S = 1 << s;
}

int freq_tile(int T, int R, int K, bool per_element);

// measured at full blocks (256, 512 and 1 024 samples); fewer samples leave
// the rest of the blocks' products unused
static double ks_rate(int K)
{
    int qb, sb, S, sl;
    ks_shape(K, qb, sb, S, sl);
    const double full = qb * sb == 1 ? 17.0 : qb * sb == 2 ? 23.0 : 25.0;
    return full * K / (256.0 * qb * sb);
}

// per path of the launch; in a per-element launch a Tx x Rx tile multiplies
// every path into all T rows (masked), the sample split only into its own
// transmitter's channels
double freq_tile_cost(int T, int R, int K, int tile, bool per_element)
{
    if (tile == 1) {
        if (K > FQ_KS_KMAX) return 1e300;
        return (double)T * R * K / ks_rate(K) / (per_element ? T : 1);
    }
    for (int i = 0; i < 5; i++)
        if (FQ_TILES[i] == tile) {
            const double tp = (double)((T + tile - 1) / tile * tile), rp = (double)((R + tile - 1) / tile * tile);
            return tp * rp * K / FQ_TILE_RATE[i];
        }
    return 1e300;
}

// the direct FP32 engine's throughput in the same units (measured on the
// batched streets); the product engine pays at 1.5x that
static const double DIRECT_RATE = 9.0;

bool freq_pays(int T, int R, int K, bool per_element)
{
    const int tile = freq_tile(T, R, K, per_element);
    // useful complex multiply-adds per path: T R K (shared) or R K (per element)
    const double work = (double)T * R * K / (per_element ? T : 1);
    return work / freq_tile_cost(T, R, K, tile, per_element) >= 1.5 * DIRECT_RATE;
}

int freq_tile(int T, int R, int K, bool per_element)
{
    int best = 96;
    for (int tile : {1, 16, 32, 48, 64, 96})
        if (freq_tile_cost(T, R, K, tile, per_element) < freq_tile_cost(T, R, K, best, per_element))
            best = tile;
    return best;
}

bool freq_own_tx(int tile, bool per_element, bool has_groups)
{
    return tile == 1 && per_element && has_groups;
}

int64_t freq_table_entries(int T, int R, int M, int64_t Ppad, bool own_tx)
{
    return (int64_t)M * ((own_tx ? 1 : T) + R) * Ppad;
}

void freq_splits(int tile, int T, int R, int M, int K, int64_t Ppad, int &n_split, int64_t &split_len)
{
    // enough workgroups to fill the chip four times over (one per CU at a
    // time), at least 16 steps of paths each
    int64_t groups;
    if (tile == 1) {
        groups = ((int64_t)M * T * R + FQ_G - 1) / FQ_G;
    } else {
        const int64_t kg = (K + FQ_G - 1) / FQ_G;
        groups = (int64_t)M * kg * ((T + tile - 1) / tile) * ((R + tile - 1) / tile);
    }
    int64_t ns = std::max<int64_t>(1, (1024 + groups - 1) / groups);
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, Ppad / (16 * FQ_PAD)));
    int64_t len = (Ppad + ns - 1) / ns;
    len = (len + FQ_PAD - 1) / FQ_PAD * FQ_PAD;
    n_split = (int)((Ppad + len - 1) / len);
    split_len = len;
}

hipError_t launch_freq_gemm(const uint2 *xt, const uint2 *yt, const float *amp, const int32_t *src,
                            int T, int R, int M, int K, int64_t Ppad, int n_split, int64_t split_len,
                            int per_element, int tile, const int64_t *rng_lo, const int64_t *rng_hi,
                            const int64_t *groups, float2 *partial, float2 *cube, hipStream_t s)
{
    if ((int64_t)n_split * split_len < Ppad || split_len % FQ_PAD || Ppad % FQ_PAD || Ppad <= 0)
        return hipErrorInvalidValue;
    if (tile != 1 && tile != 16 && tile != 32 && tile != 48 && tile != 64 && tile != 96)
        return hipErrorInvalidValue;
    if (tile == 1 && K > FQ_KS_KMAX) return hipErrorInvalidValue;
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
    A.tt = (T + tile - 1) / tile;
    A.rt = (R + tile - 1) / tile;
    A.kg = (K + FQ_G - 1) / FQ_G;
    A.n_split = n_split;
    A.split_len = split_len;
    A.partial = n_split > 1;
    A.out = n_split > 1 ? partial : cube;
    A.rng_lo = rng_lo;
    A.rng_hi = rng_hi;
    A.groups = tile == 1 && per_element ? groups : nullptr;
    int qb = 1, sb = 1;
    ks_shape(K, qb, sb, A.S, A.S_log2);
    A.n_waves = (int64_t)n_split * M * T * R;
    const int64_t blocks = tile == 1 ? (A.n_waves + FQ_G - 1) / FQ_G
                                     : (int64_t)n_split * M * A.tt * A.rt * A.kg;
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const dim3 g((unsigned)blocks), t(FQ_G * 64);
    const bool pe = per_element != 0;
#define KS_LAUNCH(QB, SB)                                                                         \
    do {                                                                                          \
        if (pe) hipLaunchKernelGGL((k_freq_ks<true, QB, SB>), g, t, 0, s, A);                     \
        else hipLaunchKernelGGL((k_freq_ks<false, QB, SB>), g, t, 0, s, A);                       \
    } while (0)
#define FQ_LAUNCH(BS, NB)                                                                         \
    do {                                                                                          \
        if (pe) hipLaunchKernelGGL((k_freq_gemm<true, BS, NB>), g, t, 0, s, A);                   \
        else hipLaunchKernelGGL((k_freq_gemm<false, BS, NB>), g, t, 0, s, A);                     \
    } while (0)
    switch (tile) {
    case 1:
        if (qb == 1 && sb == 1) KS_LAUNCH(1, 1);
        else if (qb == 1) KS_LAUNCH(1, 2);
        else KS_LAUNCH(2, 2);
        break;
    case 16: FQ_LAUNCH(16, 1); break;
    case 48: FQ_LAUNCH(16, 3); break;
    case 32: FQ_LAUNCH(32, 1); break;
    case 64: FQ_LAUNCH(32, 2); break;
    default: FQ_LAUNCH(32, 3); break;
    }
#undef FQ_LAUNCH
#undef KS_LAUNCH
    if (n_split > 1) {
        const int64_t per = (int64_t)M * K * T * R;
        hipLaunchKernelGGL(k_freq_reduce, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, s,
                           partial, n_split, T, R, M, K, cube);
    }
    return hipGetLastError();
}
