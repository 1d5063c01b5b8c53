// k_mlp.hip -- the learned ray proposal: scene probe, training histogram,
// a 4-layer MLP (18 -> 64 -> 64 -> 64 -> 1, ReLU) with forward, backward and
// Adam kernels, and the sampling table (softmax mixed with the uniform density,
// then its CDF) that the tracer's importance sampler reads.
//
// Weights and activations are stored in FP16; every product is formed and
// accumulated in FP32 (an FP16 x FP16 product is exact in FP32).  Every layer
// runs on the matrix cores: the forward pass in FP16 MFMA, the backward pass
// and the weight gradients in FP32 MFMA (the gradients fall below FP16's
// normal range), 32 rows per wavefront; the weight gradients are reduced in
// a fixed order.
#include <hip/hip_fp16.h>

#include "rr_internal.h"

namespace {

#define NAZ 128
#define NEL 64
#define NBINS (NAZ * NEL)
#define NIN 18
#define NH 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + NH * NIN)
#define OFF_W2 (OFF_B1 + NH)
#define OFF_B2 (OFF_W2 + NH * NH)
#define OFF_W3 (OFF_B2 + NH)
#define OFF_B3 (OFF_W3 + NH * NH)
#define OFF_W4 (OFF_B3 + NH)
#define OFF_B4 (OFF_W4 + NH)
#define NPARAMS (OFF_B4 + 1)

static_assert(NPARAMS == RR_MLP_PARAMS, "parameter count");

__device__ __forceinline__ float h16(float x) { return __half2float(__float2half(x)); }

// input k of row r: k = 0, 1 the bin's azimuth and elevation centre mapped
// to [-1, 1], k = 2 .. 17 the scene code (all rounded to FP16)
__device__ __forceinline__ float row_input_k(const float *codes, int64_t r, int k)
{
    const int64_t s = r / NBINS;
    const int b = (int)(r - s * NBINS);
    if (k == 0) return h16(2.0f * ((float)(b % NAZ) + 0.5f) / (float)NAZ - 1.0f);
    if (k == 1) return h16(2.0f * ((float)(b / NAZ) + 0.5f) / (float)NEL - 1.0f);
    return h16(codes[s * 16 + k - 2]);
}

// forward on the matrix cores (v_mfma_f32_32x32x16_f16: FP16 operands, FP32
// accumulation; an FP16 x FP16 product is exact in FP32).  A wavefront takes
// 32 rows: per hidden layer the activations (32 x 64, FP16) are the A operand
// and the weights the B operand (in x out, 16 inputs a step; layer 1's 18
// inputs padded to 32 with zeros), then bias, ReLU and the FP16 rounding in
// FP32 on the accumulators; the activations go through LDS (row-major) to
// become the next layer's A fragments.  Logit: each of lanes 0..31 takes its
// row's dot product with W4 in input order.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
#define MF_RS (NH + 8)              // LDS row stride of an activation tile (halves)
#define MF_FRAGS (2 * 2 + 2 * 4 * 2)  // B fragments: layer 1 (2 column blocks x 2 input steps), layers 2, 3 (2 x 4 each)

// B fragment (column block cb, input step kc) of a layer with weights
// w[out][in] (in-width nin): lane l holds output 32 cb + l % 32, inputs
// 16 kc + 8 (l / 32) .. + 7, rounded to FP16 (zero beyond nin)
__device__ __forceinline__ uint4 wfrag(const float *w, int nin, int cb, int kc, int l)
{
    const int j = 32 * cb + (l & 31), i0 = 16 * kc + 8 * (l >> 5);
    f16x8 v;
#pragma unroll
    for (int e = 0; e < 8; e++) v[e] = (_Float16)(i0 + e < nin ? w[j * nin + i0 + e] : 0.0f);
    return __builtin_bit_cast(uint4, v);
}

__global__ __launch_bounds__(256) void k_mlp_fwd(const float *P, const float *codes, int64_t n,
                                                 __half *acts, float *z)
{
    __shared__ uint4 Wf[MF_FRAGS][64];
    __shared__ float Bs[3][NH], W4s[NH + 1];
    __shared__ _Float16 Hs[4][32][MF_RS];
    for (int q = threadIdx.x; q < MF_FRAGS * 64; q += blockDim.x) {
        const int f = q >> 6, l = q & 63;
        uint4 v;
        if (f < 4) v = wfrag(P + OFF_W1, NIN, f >> 1, f & 1, l);
        else if (f < 12) v = wfrag(P + OFF_W2, NH, (f - 4) >> 2, (f - 4) & 3, l);
        else v = wfrag(P + OFF_W3, NH, (f - 12) >> 2, (f - 12) & 3, l);
        Wf[f][l] = v;
    }
    for (int q = threadIdx.x; q < NH; q += blockDim.x) {
        Bs[0][q] = h16(P[OFF_B1 + q]);
        Bs[1][q] = h16(P[OFF_B2 + q]);
        Bs[2][q] = h16(P[OFF_B3 + q]);
        W4s[q] = h16(P[OFF_W4 + q]);
    }
    if (threadIdx.x == 0) W4s[NH] = h16(P[OFF_B4]);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * 32;
    if (r0 >= n) return;
    const int row = lane & 31, half = lane >> 5;
    const int64_t r = r0 + row;
    const bool live = r < n;
    _Float16(*H)[MF_RS] = Hs[w];

    // layer-1 A fragments: inputs 8 half .. + 7 (step 0) and 16 + 8 half .. (step 1)
    uint4 A[4];
    {
        f16x8 a0, a1;
#pragma unroll
        for (int e = 0; e < 8; e++) {
            a0[e] = (_Float16)row_input_k(codes, live ? r : n - 1, 8 * half + e);
            a1[e] = (_Float16)(!half && e < NIN - 16 ? row_input_k(codes, live ? r : n - 1, 16 + e) : 0.0f);
        }
        A[0] = __builtin_bit_cast(uint4, a0);
        A[1] = __builtin_bit_cast(uint4, a1);
    }
#pragma unroll
    for (int L = 0; L < 3; L++) {
        const int nk = L == 0 ? 2 : 4;                   // input steps of the layer
        const int fb = L == 0 ? 0 : (L == 1 ? 4 : 12);   // its first B fragment
        f32x16 acc[2];
#pragma unroll
        for (int cb = 0; cb < 2; cb++) {
#pragma unroll
            for (int e = 0; e < 16; e++) acc[cb][e] = 0.0f;
#pragma unroll
            for (int kc = 0; kc < 4; kc++)
                if (kc < nk)
                    acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                        __builtin_bit_cast(f16x8, A[kc]),
                        __builtin_bit_cast(f16x8, Wf[fb + cb * nk + kc][lane]), acc[cb], 0, 0, 0);
        }
        // D layout: register e of lane l is row 8 (e / 4) + 4 (l / 32) + e % 4,
        // column l % 32 of the block
#pragma unroll
        for (int cb = 0; cb < 2; cb++) {
            const int j = 32 * cb + (lane & 31);
            const float bj = Bs[L][j];
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int rr = 8 * (e >> 2) + 4 * half + (e & 3);
                H[rr][j] = (_Float16)fmaxf(acc[cb][e] + bj, 0.0f);
            }
        }
        // the wavefront's own tile: its LDS operations run in order
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int kc = 0; kc < 4; kc++) A[kc] = *reinterpret_cast<const uint4 *>(&H[row][16 * kc + 8 * half]);
        if (acts && live) {
#pragma unroll
            for (int kc = 0; kc < 4; kc++)
                *reinterpret_cast<uint4 *>(acts + ((int64_t)L * n + r) * NH + 16 * kc + 8 * half) = A[kc];
        }
    }
    if (half == 0 && live) {
        float a = W4s[NH];
#pragma unroll
        for (int i = 0; i < NH; i++) a = fmaf(W4s[i], (float)H[row][i], a);
        z[r] = a;
    }
}

// per scene: softmax of the logits; loss -sum H log q / sum H and its
// gradient dz = (q - H / sum H) / n_scenes (zero for a scene with no target)
__global__ __launch_bounds__(1024) void k_softmax_grad(const float *z, const float *H, int n_scenes,
                                                       float *dz, float *loss)
{
    __shared__ float red[1024];
    const int s = blockIdx.x;
    const float *zs = z + (int64_t)s * NBINS;
    const float *hs = H + (int64_t)s * NBINS;
    float mx = -3.0e38f, hsum = 0.0f;
    for (int b = threadIdx.x; b < NBINS; b += 1024) {
        mx = fmaxf(mx, zs[b]);
        hsum += hs[b];
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    mx = red[0];
    __syncthreads();
    float es = 0.0f;
    for (int b = threadIdx.x; b < NBINS; b += 1024) es += __expf(zs[b] - mx);
    red[threadIdx.x] = es;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const float lse = logf(red[0]);
    __syncthreads();
    red[threadIdx.x] = hsum;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const float Hs = red[0];
    __syncthreads();
    float l = 0.0f;
    for (int b = threadIdx.x; b < NBINS; b += 1024) {
        const float logq = zs[b] - mx - lse;
        float d = 0.0f;
        if (Hs > 0.0f) {
            l -= hs[b] * logq;
            d = (__expf(logq) - hs[b] / Hs) / (float)n_scenes;
        }
        dz[(int64_t)s * NBINS + b] = d;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[s] = Hs > 0.0f ? red[0] / Hs / (float)n_scenes : 0.0f;
}

// Backward pass on the matrix cores in FP32 (v_mfma_f32_32x32x2f32): the
// gradients fall below FP16's normal range, so they stay FP32 throughout.
// A wavefront takes 32 rows: d3 = [h3 > 0] dz W4 (vector units), then
// d2 = [h2 > 0] (d3 W3) and d1 = [h1 > 0] (d2 W2) as (32 x 64) by (64 x 64)
// products, the weights (FP16-rounded) as the B operand from LDS and the
// previous gradient tile as the A operand from LDS (row-major, one float a
// lane and step); every gradient tile is also written out for the weight
// gradients.
#define BW_RS (NH + 1)
__global__ __launch_bounds__(256) void k_mlp_bwd(const float *P, const float *dz, int64_t n,
                                                 const __half *acts, float *d1, float *d2, float *d3)
{
    __shared__ _Float16 Ws[2][NH][NH];     // W3, W2 as [out j][in i] (FP16 values: exact)
    __shared__ float W4s[NH];
    __shared__ float Dt[4][32][BW_RS];
    for (int q = threadIdx.x; q < NH * NH; q += blockDim.x) {
        Ws[0][q / NH][q % NH] = (_Float16)P[OFF_W3 + q];
        Ws[1][q / NH][q % NH] = (_Float16)P[OFF_W2 + q];
    }
    for (int q = threadIdx.x; q < NH; q += blockDim.x) W4s[q] = h16(P[OFF_W4 + q]);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * 32;
    if (r0 >= n) return;
    const int rows = (int)min((int64_t)32, n - r0);
    float(*D)[BW_RS] = Dt[w];
    // d3: lane j over the tile's rows (coalesced)
    {
        const int j = lane;
#pragma unroll 8
        for (int rr = 0; rr < 32; rr++) {
            float v = 0.0f;
            if (rr < rows) {
                const int64_t r = r0 + rr;
                v = __half2float(acts[(2 * n + r) * NH + j]) > 0.0f ? dz[r] * W4s[j] : 0.0f;
                d3[r * NH + j] = v;
            }
            D[rr][j] = v;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const int col = lane & 31, kk = lane >> 5;
#pragma unroll
    for (int L = 0; L < 2; L++) {
        // out[r][i] = sum_j D[r][j] W[j][i]: A[r][k = j] = D, B[k = j][i] = W
        f32x16 acc[2];
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int e = 0; e < 16; e++) acc[cb][e] = 0.0f;
#pragma unroll 8
        for (int ks = 0; ks < NH / 2; ks++) {
            const int k = 2 * ks + kk;
            const float av = D[col][k];
#pragma unroll
            for (int cb = 0; cb < 2; cb++)
                acc[cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, (float)Ws[L][k][32 * cb + col], acc[cb], 0, 0, 0);
        }
        const __half *h = acts + (int64_t)(1 - L) * n * NH;
        float *dout = L == 0 ? d2 : d1;
        __builtin_amdgcn_wave_barrier();
        // D layout: register e of lane l is row 8 (e / 4) + 4 (l / 32) + e % 4,
        // column l % 32 of the block
#pragma unroll
        for (int cb = 0; cb < 2; cb++) {
            const int i = 32 * cb + col;
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int rr = 8 * (e >> 2) + 4 * kk + (e & 3);
                float v = 0.0f;
                if (rr < rows) {
                    const int64_t r = r0 + rr;
                    v = __half2float(h[r * NH + i]) > 0.0f ? acc[cb][e] : 0.0f;
                    dout[r * NH + i] = v;
                }
                D[rr][i] = v;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Weight gradients on the matrix cores in FP32 (v_mfma_f32_32x32x2f32):
//   G[a][c] = sum_r D[r][a] V[r][c],  Gb[a] = sum_r D[r][a]
// as (da x rows) by (rows x vc) products, two rows a step: lane l takes
// D[r + l / 32][a] and V[r + l / 32][c] for a, c = l % 32 (+ 32) straight from
// memory (coalesced).  V is the FP16 activation (width 64) or, without it,
// the layer-1 input (width 18, rebuilt from the bin and the scene code).
// Block b sums its rows in order and writes its partial sums to row b of the
// partial table (stride NPARAMS, at the layer's parameter offsets); two
// passes then add the rows in a fixed order, so the gradient is the same
// bits on every run.
#define WG_MAXB 4096      // most blocks (partial-table rows) per layer
#define WG_MINR 64        // fewest rows per block
#define WG_RUN 32         // rows of the partial table added per first-pass run
#define WG_STEPS 8        // two-row steps loaded together
__global__ __launch_bounds__(64) void k_wgrad(const float *D, int da, const __half *V,
                                              const float *codes, int vc, int64_t n,
                                              int64_t rows_per_block, float *part, int off_g,
                                              int off_b)
{
    float *G = part + (int64_t)blockIdx.x * NPARAMS + off_g;
    float *Gb = part + (int64_t)blockIdx.x * NPARAMS + off_b;
    const int lane = threadIdx.x, col = lane & 31, kk = lane >> 5;
    const int nab = da > 32 ? 2 : 1, ncb = vc > 32 ? 2 : 1;
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) acc[i][j][e] = 0.0f;
    float bs[2] = {0.0f, 0.0f};
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(n, r0 + rows_per_block);
    // WG_STEPS steps (two rows each) at a time, the next group's values
    // loaded while this group's products run
    float ca[WG_STEPS][2], cv[WG_STEPS][2], na[WG_STEPS][2], nv[WG_STEPS][2];
    auto load = [&](int64_t rbase, float (&xa)[WG_STEPS][2], float (&xv)[WG_STEPS][2]) {
#pragma unroll
        for (int q = 0; q < WG_STEPS; q++) {
            const int64_t row = rbase + 2 * q + kk;
            const bool ok = row < r1;
#pragma unroll
            for (int i = 0; i < 2; i++) {
                const int a = 32 * i + col;
                xa[q][i] = ok && i < nab && a < da ? D[row * da + a] : 0.0f;
                const int c = 32 * i + col;
                xv[q][i] = 0.0f;
                if (ok && i < ncb && c < vc)
                    xv[q][i] = V ? __half2float(V[row * vc + c]) : row_input_k(codes, row, c);
            }
        }
    };
    load(r0, ca, cv);
    for (int64_t rb = r0; rb < r1; rb += 2 * WG_STEPS) {
        if (rb + 2 * WG_STEPS < r1) load(rb + 2 * WG_STEPS, na, nv);
#pragma unroll
        for (int q = 0; q < WG_STEPS; q++)
#pragma unroll
            for (int i = 0; i < 2; i++) {
                bs[i] += ca[q][i];
#pragma unroll
                for (int j = 0; j < 2; j++)
                    if (i < nab && j < ncb)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[q][i], cv[q][j], acc[i][j], 0, 0, 0);
            }
#pragma unroll
        for (int q = 0; q < WG_STEPS; q++)
#pragma unroll
            for (int i = 0; i < 2; i++) {
                ca[q][i] = na[q][i];
                cv[q][i] = nv[q][i];
            }
    }
    // D layout: register e of lane l is row (a) 8 (e / 4) + 4 (l / 32) + e % 4,
    // column (c) l % 32 of the block
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 16; e++) {
                const int a = 32 * i + 8 * (e >> 2) + 4 * kk + (e & 3), c = 32 * j + col;
                if (i < nab && j < ncb && a < da && c < vc) G[a * vc + c] = acc[i][j][e];
            }
    // bias: the even rows' sum (lanes 0..31) plus the odd rows' (lanes 32..63)
#pragma unroll
    for (int i = 0; i < 2; i++) {
        const float other = __shfl_down(bs[i], 32, 64);
        const int a = 32 * i + col;
        if (kk == 0 && i < nab && a < da) Gb[a] = bs[i] + other;
    }
}

// first pass: run y of the partial table (rows y WG_RUN .. + WG_RUN - 1, in
// order) into row nb + y; second pass: those runs in order into G
__global__ __launch_bounds__(256) void k_wgrad_sum(float *part, int nb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAMS) return;
    const int y = blockIdx.y;
    const int b0 = y * WG_RUN, b1 = min(nb, b0 + WG_RUN);
    float s = 0.0f;
    for (int b = b0; b < b1; b++) s += part[(int64_t)b * NPARAMS + i];
    part[(int64_t)(nb + y) * NPARAMS + i] = s;
}

__global__ __launch_bounds__(256) void k_wgrad_sum2(const float *part, int nb, int runs, float *G)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAMS) return;
    float s = 0.0f;
    for (int y = 0; y < runs; y++) s += part[(int64_t)(nb + y) * NPARAMS + i];
    G[i] = s;
}

// Adam (Kingma & Ba): FP32 master parameters and moments
__global__ void k_adam(float *P, const float *G, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// sampling table for one scene: q_mix = (1 - beta) d / sum d + beta / NBINS
// with d = exp(power z) (kappa = 0: the softmax of power z), or, with kappa >
// 0, d = sqrt(x / (kappa + x)) where x = NBINS softmax(z) is a bin's fitted
// return density relative to the mean (the density of least variance x cost
// when a ray costs kappa mean returns); cdf[0] = 0, cdf[b + 1] = cdf[b] +
// q_mix[b] (FP64, block scan), normalised
__global__ __launch_bounds__(1024) void k_build_cdf(const float *z, float beta, float power,
                                                    float kappa, double *cdf)
{
    __shared__ double red[1024];
    __shared__ float fred[1024];
    const int t = threadIdx.x;
    float mx = -3.0e38f;
    for (int b = t; b < NBINS; b += 1024) mx = fmaxf(mx, z[b]);
    fred[t] = mx;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) fred[t] = fmaxf(fred[t], fred[t + o]);
        __syncthreads();
    }
    mx = fred[0];
    __syncthreads();
    // each thread owns 8 consecutive bins
    const double pw = kappa > 0.0f ? 1.0 : (double)power;
    double e[8];
    double s = 0.0;
    for (int k = 0; k < 8; k++) {
        e[k] = exp(pw * ((double)z[t * 8 + k] - (double)mx));
        s += e[k];
    }
    red[t] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    double tot = red[0];
    __syncthreads();
    if (kappa > 0.0f) {
        // x = NBINS e / tot; d = sqrt(x / (kappa + x)); then normalise d
        double s2 = 0.0;
        for (int k = 0; k < 8; k++) {
            const double x = (double)NBINS * e[k] / tot;
            e[k] = sqrt(x / ((double)kappa + x));
            s2 += e[k];
        }
        red[t] = s2;
        __syncthreads();
        for (int o = 512; o > 0; o >>= 1) {
            if (t < o) red[t] += red[t + o];
            __syncthreads();
        }
        tot = red[0];
        __syncthreads();
    }
    double loc = 0.0;
    double q[8];
    for (int k = 0; k < 8; k++) {
        q[k] = (1.0 - (double)beta) * e[k] / tot + (double)beta / (double)NBINS;
        loc += q[k];
    }
    // inclusive scan of per-thread sums (Hillis-Steele)
    red[t] = loc;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        double y = t >= o ? red[t - o] : 0.0;
        __syncthreads();
        red[t] += y;
        __syncthreads();
    }
    const double total = red[1023];
    double run = red[t] - loc;
    for (int k = 0; k < 8; k++) {
        run += q[k];
        cdf[t * 8 + k + 1] = run / total;
    }
    if (t == 0) cdf[0] = 0.0;
    __syncthreads();
    if (t == 1023) cdf[NBINS] = 1.0;
}

}  // namespace

hipError_t launch_mlp_forward(const float *P, const float *codes, int64_t n, __half *acts, float *z,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((n + 127) / 128)), dim3(256), 0, s, P, codes, n,
                       acts, z);
    return hipGetLastError();
}

hipError_t launch_softmax_grad(const float *z, const float *H, int n_scenes, float *dz, float *loss,
                               hipStream_t s)
{
    if (n_scenes <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_softmax_grad, dim3(n_scenes), dim3(1024), 0, s, z, H, n_scenes, dz, loss);
    return hipGetLastError();
}

// blocks of the weight-gradient kernels: an even number of rows each, at
// least WG_MINR (small batches keep a small partial table), at most WG_MAXB
// blocks
static int wgrad_blocks(int64_t n, int64_t &rows_per_block)
{
    int64_t rpb = (n + WG_MAXB - 1) / WG_MAXB;
    rpb = std::max<int64_t>(WG_MINR, (rpb + 1) / 2 * 2);
    rows_per_block = rpb;
    return (int)((n + rpb - 1) / rpb);
}

int64_t mlp_part_rows(int64_t n)
{
    int64_t rpb;
    const int nb = wgrad_blocks(std::max<int64_t>(n, 1), rpb);
    return nb + (nb + WG_RUN - 1) / WG_RUN;
}

hipError_t launch_mlp_backward(const float *P, const float *dz, int64_t n, const __half *acts,
                               float *d1, float *d2, float *d3, const float *codes, float *part,
                               float *grad, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)((n + 127) / 128)), dim3(256), 0, s, P, dz, n, acts,
                       d1, d2, d3);
    int64_t rpb;
    const int nb = wgrad_blocks(n, rpb);
    // layer 4: dz (width 1) x h3; layer 3: d3 x h2; layer 2: d2 x h1; layer 1: d1 x input
    hipLaunchKernelGGL(k_wgrad, dim3(nb), dim3(64), 0, s, dz, 1, acts + 2 * n * NH, codes, NH, n, rpb,
                       part, OFF_W4, OFF_B4);
    hipLaunchKernelGGL(k_wgrad, dim3(nb), dim3(64), 0, s, d3, NH, acts + 1 * n * NH, codes, NH, n, rpb,
                       part, OFF_W3, OFF_B3);
    hipLaunchKernelGGL(k_wgrad, dim3(nb), dim3(64), 0, s, d2, NH, acts + 0 * n * NH, codes, NH, n, rpb,
                       part, OFF_W2, OFF_B2);
    hipLaunchKernelGGL(k_wgrad, dim3(nb), dim3(64), 0, s, d1, NH, (const __half *)nullptr, codes, NIN,
                       n, rpb, part, OFF_W1, OFF_B1);
    const int runs = (nb + WG_RUN - 1) / WG_RUN;
    hipLaunchKernelGGL(k_wgrad_sum, dim3((NPARAMS + 255) / 256, runs), dim3(256), 0, s, part, nb);
    hipLaunchKernelGGL(k_wgrad_sum2, dim3((NPARAMS + 255) / 256), dim3(256), 0, s, part, nb, runs, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float *P, const float *G, float *m, float *v, float lr, int step, hipStream_t s)
{
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((NPARAMS + 255) / 256), dim3(256), 0, s, P, G, m, v, NPARAMS, lr,
                       b1, b2, 1e-8f, c1, c2);
    return hipGetLastError();
}

hipError_t launch_build_cdf(const float *z, float beta, float power, float kappa, double *cdf,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_build_cdf, dim3(1), dim3(1024), 0, s, z, beta, power, kappa, cdf);
    return hipGetLastError();
}
