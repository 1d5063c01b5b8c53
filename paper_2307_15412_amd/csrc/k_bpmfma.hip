// k_bpmfma.hip -- delay-and-sum back-projection on the matrix cores.
//
// image(x) = sum_n sum_t a_t(n) sum_r S_n[t, r] b_r(n),
//     a_t(n) = exp(+j 2 pi f_n |x - tx_t| / c),  b_r(n) = exp(+j 2 pi f_n |x - rx_r| / c),
// because the two legs of the delay add: the inner sum over receivers is, for
// every frequency, the complex product of the cube slice S_n (Tx x Rx) with
// the matrix of receive phasors of a block of voxels (Rx x voxels), the same
// multiply-adds as the brute-force sum.  A workgroup of eight wavefronts (two
// per SIMD) owns 128 voxels, 16 per wavefront; per frequency each wavefront
// computes U = S_n B (96 x 16 over 96 receivers: six 16 x 16 blocks, three
// 32-receiver steps, split bf16 hi + lo, 216 v_mfma_f32_16x16x32_bf16) and
// adds sum_t a_t U[t, voxel] on the vector units; the two wavefronts of a SIMD
// overlap one's phasor work with the other's products.  S_n, prepared once in
// the A-operand fragment layout, is double-buffered in LDS and loaded by LDS
// DMA one frequency ahead.  Leg lengths are formed in FP64 once per voxel and
// kept in FP32 (the phase f d / c stays below 256 turns in an imaging volume
// of a few tens of centimetres, where FP32 keeps it to ~1e-5 turn); the
// hardware sin/cos take turns.  Needs at most 96 transmitters and receivers.
#include "rr_internal.h"

namespace {

#define BG_W 8                 // wavefronts per workgroup
#define BG_VW 16               // voxels per wavefront
#define BG_TB 6                // 16-row Tx blocks
#define BG_RS 3                // 32-receiver steps
#define BG_NF (BG_TB * BG_RS * 4)   // 1 KiB fragments per frequency (4 planes)

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned pack_bf16(float x, float y)
{
    f32x2 v = {x, y};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ void split_bf16(float x, float y, unsigned &hi, unsigned &lo)
{
    hi = pack_bf16(x, y);
    lo = pack_bf16(x - __uint_as_float(hi << 16), y - __uint_as_float(hi & 0xffff0000u));
}

__device__ __forceinline__ bf16x8 as_bf(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ uint4 neg(uint4 v)
{
    return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u, v.w ^ 0x80008000u);
}

#define MFMA(a, b, c) __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a), as_bf(b), c, 0, 0, 0)

// Cube slices in the A-operand layout of the 16 x 16 x 32 product: fragment
// (n, tb, rs, plane) lane l holds S_n[16 tb + l % 16][32 rs + 8 (l / 16) + e],
// e = 0..7, as bf16; planes: real hi, real lo, imaginary hi, imaginary lo;
// zero outside T x R.
__global__ void k_bp_prep(const float2 *cube, int64_t stride, int T, int R, int K, uint4 *Sf)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)K * BG_TB * BG_RS * 64) return;
    const int lane = (int)(g & 63);
    int64_t f = g >> 6;
    const int rs = (int)(f % BG_RS);
    f /= BG_RS;
    const int tb = (int)(f % BG_TB);
    const int n = (int)(f / BG_TB);
    const int t = tb * 16 + (lane & 15);
    const int r0 = rs * 32 + (lane >> 4) * 8;
    float re[8], im[8];
    for (int e = 0; e < 8; e++) {
        float2 v = make_float2(0.0f, 0.0f);
        if (t < T && r0 + e < R) v = cube[((int64_t)t * R + r0 + e) * stride + n];
        re[e] = v.x;
        im[e] = v.y;
    }
    uint4 p[4];
    unsigned *rh = &p[0].x, *rl = &p[1].x, *ih = &p[2].x, *il = &p[3].x;
    for (int q = 0; q < 4; q++) {
        split_bf16(re[2 * q], re[2 * q + 1], rh[q], rl[q]);
        split_bf16(im[2 * q], im[2 * q + 1], ih[q], il[q]);
    }
    const int64_t base = ((((int64_t)n * BG_TB + tb) * BG_RS + rs) * 4) * 64 + lane;
    for (int q = 0; q < 4; q++) Sf[base + q * 64] = p[q];
}

__device__ __forceinline__ double dist3(double x, double y, double z, const double *p)
{
    const double dx = x - p[0], dy = y - p[1], dz = z - p[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

struct BpMfmaArgs {
    const uint4 *Sf;
    const double *tx, *rx;
    int T, R, K;
    double f0, df, inv_c;
    double x0, y0, z0, step;
    int nx, ny, nz;
    int64_t n_vox;
    float2 *image;
};

__global__ __launch_bounds__(BG_W * 64) void k_bp_mfma(BpMfmaArgs A)
{
    __shared__ uint4 Ss[2][BG_NF * 64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q4 = lane >> 4;
    const int64_t v = (int64_t)blockIdx.x * (BG_W * BG_VW) + w * BG_VW + (lane & 15);
    const bool valid = v < A.n_vox;
    const int64_t plane = (int64_t)A.ny * A.nz;
    const int64_t vv = valid ? v : 0;
    const int i = (int)(vv / plane);
    const int64_t rem = vv - (int64_t)i * plane;
    const int j = (int)(rem / A.nz), k = (int)(rem - (int64_t)j * A.nz);
    const double x = A.x0 + (double)i * A.step, y = A.y0 + (double)j * A.step,
                 z = A.z0 + (double)k * A.step;
    // this lane's legs: the Tx rows of its accumulator elements (16 tb + 4 q4
    // + e) and the Rx rows of its B-operand slots (32 rs + 8 q4 + e)
    float dt[BG_TB * 4], dr[BG_RS * 8];
#pragma unroll
    for (int tb = 0; tb < BG_TB; tb++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int t = tb * 16 + 4 * q4 + e;
            dt[tb * 4 + e] = t < A.T ? (float)dist3(x, y, z, A.tx + 3 * t) : 0.0f;
        }
#pragma unroll
    for (int rs = 0; rs < BG_RS; rs++)
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int r = rs * 32 + 8 * q4 + e;
            dr[rs * 8 + e] = r < A.R ? (float)dist3(x, y, z, A.rx + 3 * r) : 0.0f;
        }
    // LDS DMA of one frequency's 72 fragments: 9 per wavefront
    auto fetch = [&](int n, int buf) {
        const uint4 *src = A.Sf + (int64_t)n * (BG_NF * 64) + lane;
#pragma unroll
        for (int q = 0; q < BG_NF / BG_W; q++) {
            const int c = w * (BG_NF / BG_W) + q;
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void *)(src + c * 64),
                (__attribute__((address_space(3))) void *)(&Ss[buf][c * 64]), 16, 0, 0);
        }
    };
    float img_re = 0.0f, img_im = 0.0f;
    // the B operands of one frequency: receive phasors of this lane's voxel
    // for its 24 receiver slots, split into six bf16 planes per step
    struct BOps {
        uint4 rh[BG_RS], rl[BG_RS], ih[BG_RS], il[BG_RS], nih[BG_RS], nil[BG_RS];
    };
    auto gen_b = [&](float fc, BOps &b) {
#pragma unroll
        for (int rs = 0; rs < BG_RS; rs++) {
            float br[8], bi[8];
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const float ph = dr[rs * 8 + e] * fc;
                br[e] = __builtin_amdgcn_cosf(ph);
                bi[e] = __builtin_amdgcn_sinf(ph);
            }
            unsigned *prh = &b.rh[rs].x, *prl = &b.rl[rs].x, *pih = &b.ih[rs].x, *pil = &b.il[rs].x;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                split_bf16(br[2 * q], br[2 * q + 1], prh[q], prl[q]);
                split_bf16(bi[2 * q], bi[2 * q + 1], pih[q], pil[q]);
            }
            b.nih[rs] = neg(b.ih[rs]);
            b.nil[rs] = neg(b.il[rs]);
        }
    };
    auto freq = [&](int n) { return (float)((A.f0 + (double)n * A.df) * A.inv_c); };
    // The two wavefronts of a SIMD run skewed: the leading half (w >= 4)
    // makes the next frequency's B operands after its Tx sum, so it starts
    // each frequency with matrix products while the other half is still
    // generating phasors, and the other way round at the end.
    const bool lead = w >= BG_W / 2;
    BOps b;
    fetch(0, 0);
    if (lead) gen_b(freq(0), b);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const f32x4 zero = {};
    for (int n = 0; n < A.K; n++) {
        const float fc = freq(n);
        if (!lead) gen_b(fc, b);
        const uint4 *S = Ss[n & 1];
        f32x4 ur[BG_TB], ui[BG_TB];
#pragma unroll
        for (int rs = 0; rs < BG_RS; rs++) {
#pragma unroll
            for (int tb = 0; tb < BG_TB; tb++) {
                const int fb = ((tb * BG_RS + rs) * 4) * 64 + lane;
                const uint4 Srh = S[fb], Srl = S[fb + 64], Sih = S[fb + 128], Sil = S[fb + 192];
                // U_re += Sr Br - Si Bi, U_im += Sr Bi + Si Br (hi*hi + hi*lo + lo*hi)
                ur[tb] = MFMA(Srh, b.rh[rs], rs == 0 ? zero : ur[tb]);
                ur[tb] = MFMA(Srh, b.rl[rs], ur[tb]);
                ur[tb] = MFMA(Srl, b.rh[rs], ur[tb]);
                ur[tb] = MFMA(Sih, b.nih[rs], ur[tb]);
                ur[tb] = MFMA(Sih, b.nil[rs], ur[tb]);
                ur[tb] = MFMA(Sil, b.nih[rs], ur[tb]);
                ui[tb] = MFMA(Srh, b.ih[rs], rs == 0 ? zero : ui[tb]);
                ui[tb] = MFMA(Srh, b.il[rs], ui[tb]);
                ui[tb] = MFMA(Srl, b.ih[rs], ui[tb]);
                ui[tb] = MFMA(Sih, b.rh[rs], ui[tb]);
                ui[tb] = MFMA(Sih, b.rl[rs], ui[tb]);
                ui[tb] = MFMA(Sil, b.rh[rs], ui[tb]);
            }
        }
        // every wavefront has read this frequency's slice: the next one may
        // be requested into the other buffer
        if (n + 1 < A.K) fetch(n + 1, (n + 1) & 1);
        // transmit phasors of this lane's Tx rows times U (D layout: element e
        // of lane l is row 4 (l / 16) + e, column l % 16 of each block)
#pragma unroll
        for (int tb = 0; tb < BG_TB; tb++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const float ph = dt[tb * 4 + e] * fc;
                const float ar = __builtin_amdgcn_cosf(ph), ai = __builtin_amdgcn_sinf(ph);
                img_re = fmaf(ar, ur[tb][e], fmaf(-ai, ui[tb][e], img_re));
                img_im = fmaf(ar, ui[tb][e], fmaf(ai, ur[tb][e], img_im));
            }
        if (lead && n + 1 < A.K) gen_b(freq(n + 1), b);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    // the four lanes l % 16 + 16 q hold the four quarters of one voxel's Tx rows
    img_re += __shfl_xor(img_re, 16);
    img_im += __shfl_xor(img_im, 16);
    img_re += __shfl_xor(img_re, 32);
    img_im += __shfl_xor(img_im, 32);
    if (valid && q4 == 0) A.image[v] = make_float2(img_re, img_im);
}

}  // namespace

hipError_t launch_bp_mfma(const float2 *cube, int64_t stride, const double *tx, int T,
                          const double *rx, int R, int K, double f0, double df, double inv_c,
                          double x0, double y0, double z0, double step, int nx, int ny, int nz,
                          uint4 *Sf, float2 *image, hipStream_t s)
{
    const int64_t n_vox = (int64_t)nx * ny * nz;
    if (n_vox <= 0 || K <= 0) return hipSuccess;
    if (T < 1 || R < 1 || T > BG_TB * 16 || R > BG_RS * 32) return hipErrorInvalidValue;
    const int64_t nf = (int64_t)K * BG_TB * BG_RS * 64;
    hipLaunchKernelGGL(k_bp_prep, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, s, cube, stride,
                       T, R, K, Sf);
    BpMfmaArgs A;
    A.Sf = Sf;
    A.tx = tx;
    A.rx = rx;
    A.T = T;
    A.R = R;
    A.K = K;
    A.f0 = f0;
    A.df = df;
    A.inv_c = inv_c;
    A.x0 = x0;
    A.y0 = y0;
    A.z0 = z0;
    A.step = step;
    A.nx = nx;
    A.ny = ny;
    A.nz = nz;
    A.n_vox = n_vox;
    A.image = image;
    const int64_t blocks = (n_vox + BG_W * BG_VW - 1) / (BG_W * BG_VW);
    hipLaunchKernelGGL(k_bp_mfma, dim3((unsigned)blocks), dim3(BG_W * 64), 0, s, A);
    return hipGetLastError();
}

int64_t bp_mfma_frag_bytes(int K) { return (int64_t)K * BG_NF * 64 * 16; }
