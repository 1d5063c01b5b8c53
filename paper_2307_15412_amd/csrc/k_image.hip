// k_image.hip -- delay-and-sum back-projection of a stepped-frequency cube
// and its maximum projection (the paper's imaging of the simulated data).
//
// image(x) = sum_{t, r} sum_n s[t n_rx + r][n] exp(+j 2 pi f_n d / c),
// d = |x - tx_t| + |x - rx_r|, f_n = f0 + n df: the matched filter of the
// synthesis phase.  One lane per voxel.  For each channel the two legs are
// formed in FP64 and the start phase f0 d / c and the step df d / c reduced
// modulo one cycle in FP64; the sum over frequencies, a polynomial in the step
// phasor w, is evaluated by Horner's rule in FP32,
//     S = (...((s_{K-1} w + s_{K-2}) w + s_{K-3}) ...) w + s_0,
// four fused multiply-adds per term, and the channel adds exp(+j 2 pi f0 d/c) S.
// The cube is staged through LDS in chunks of channels and read as broadcasts.
#include "rr_internal.h"

namespace {

#define BP_T 256
#define BP_SH 4096        // staged cube entries (32 KiB): 4096 / K channels per chunk

__device__ __forceinline__ double frac(double x) { return x - floor(x); }

// fixed-point turns of x modulo 1 -> FP32 turns in [-1/2, 1/2)
__device__ __forceinline__ float turns(double x)
{
    const unsigned u = (unsigned)(unsigned long long)llrint(frac(x) * 4294967296.0);
    return (float)(int)u * 2.3283064365386963e-10f;
}

__global__ __launch_bounds__(BP_T) void k_backproject(BackProjArgs A)
{
    __shared__ float2 sh[BP_SH];
    const int64_t v = (int64_t)blockIdx.x * BP_T + threadIdx.x;
    const bool valid = v < A.n_vox;
    const int64_t plane = (int64_t)A.ny * A.nz;
    const int i = valid ? (int)(v / plane) : 0;
    const int64_t rem = v - (int64_t)i * plane;
    const int j = valid ? (int)(rem / A.nz) : 0;
    const int k = valid ? (int)(rem - (int64_t)j * A.nz) : 0;
    const double x = A.x0 + (double)i * A.step, y = A.y0 + (double)j * A.step,
                 z = A.z0 + (double)k * A.step;
    const double f0c = A.f0 * A.inv_c, dfc = A.df * A.inv_c;
    const int K = A.K;
    float are = 0.0f, aim = 0.0f;
    int t = 0, r = 0;
    double dt = 0.0;
    // step phasor w = exp(+j 2 pi df d / c) and start phasor exp(+j 2 pi f0 d / c)
    // of channel (t, r); advances (t, r) to the next channel
    auto phasors = [&](int &t, int &r, double &dt, float &wr, float &wi, float &zr, float &zi) {
        if (r == 0) {
            const double ax = x - A.tx[3 * t], ay = y - A.tx[3 * t + 1], az = z - A.tx[3 * t + 2];
            dt = sqrt(ax * ax + ay * ay + az * az);
        }
        const double bx = x - A.rx[3 * r], by = y - A.rx[3 * r + 1], bz = z - A.rx[3 * r + 2];
        const double d = dt + sqrt(bx * bx + by * by + bz * bz);
        const float u0 = turns(d * f0c), u1 = turns(d * dfc);
        wr = __builtin_amdgcn_cosf(u1);
        wi = __builtin_amdgcn_sinf(u1);
        zr = __builtin_amdgcn_cosf(u0);
        zi = __builtin_amdgcn_sinf(u0);
        if (++r == A.nrx) {
            r = 0;
            t++;
        }
    };
    const int chunk = BP_SH / K;
    for (int c0 = 0; c0 < A.C; c0 += chunk) {
        const int cnt = min(chunk, A.C - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * K; e += BP_T) {
            const int cc = e / K, n = e - cc * K;
            sh[e] = A.cube[(int64_t)(c0 + cc) * A.stride + n];
        }
        __syncthreads();
        // two channels at a time: independent Horner chains for the latency
        int cc = 0;
        for (; cc + 1 < cnt; cc += 2) {
            float w0r, w0i, z0r, z0i, w1r, w1i, z1r, z1i;
            phasors(t, r, dt, w0r, w0i, z0r, z0i);
            phasors(t, r, dt, w1r, w1i, z1r, z1i);
            const float2 *s0 = sh + cc * K, *s1 = s0 + K;
            float a0r = s0[K - 1].x, a0i = s0[K - 1].y, a1r = s1[K - 1].x, a1i = s1[K - 1].y;
#pragma unroll 8
            for (int n = K - 2; n >= 0; n--) {
                const float2 q0 = s0[n], q1 = s1[n];
                const float b0r = fmaf(a0r, w0r, fmaf(-a0i, w0i, q0.x));
                const float b0i = fmaf(a0r, w0i, fmaf(a0i, w0r, q0.y));
                const float b1r = fmaf(a1r, w1r, fmaf(-a1i, w1i, q1.x));
                const float b1i = fmaf(a1r, w1i, fmaf(a1i, w1r, q1.y));
                a0r = b0r; a0i = b0i; a1r = b1r; a1i = b1i;
            }
            are = fmaf(z0r, a0r, fmaf(-z0i, a0i, are));
            aim = fmaf(z0r, a0i, fmaf(z0i, a0r, aim));
            are = fmaf(z1r, a1r, fmaf(-z1i, a1i, are));
            aim = fmaf(z1r, a1i, fmaf(z1i, a1r, aim));
        }
        for (; cc < cnt; cc++) {
            float wr, wi, zr, zi;
            phasors(t, r, dt, wr, wi, zr, zi);
            const float2 *s0 = sh + cc * K;
            float ar = s0[K - 1].x, ai = s0[K - 1].y;
#pragma unroll 8
            for (int n = K - 2; n >= 0; n--) {
                const float2 q = s0[n];
                const float br = fmaf(ar, wr, fmaf(-ai, wi, q.x));
                const float bi = fmaf(ar, wi, fmaf(ai, wr, q.y));
                ar = br; ai = bi;
            }
            are = fmaf(zr, ar, fmaf(-zi, ai, are));
            aim = fmaf(zr, ai, fmaf(zi, ar, aim));
        }
    }
    if (valid) A.image[v] = make_float2(are, aim);
}

// Maximum over range (the slowest axis) of |image|, in dB relative to the
// largest value (computed by the caller's first pass), clamped at floor_db.
__global__ void k_max_projection(const float2 *img, int64_t nx, int64_t nyz, float *out,
                                 float *peak)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nyz) return;
    float m = 0.0f;
    for (int64_t i = 0; i < nx; i++) {
        const float2 a = img[i * nyz + p];
        m = fmaxf(m, sqrtf(a.x * a.x + a.y * a.y));
    }
    out[p] = m;
    // the global maximum of non-negative floats as an unsigned integer maximum
    atomicMax(reinterpret_cast<unsigned *>(peak), __float_as_uint(m));
}

__global__ void k_to_db(float *out, int64_t nyz, const float *peak, float floor_db)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nyz) return;
    const float pk = *peak;
    float db = pk > 0.0f && out[p] > 0.0f ? 20.0f * log10f(out[p] / pk) : floor_db;
    out[p] = fmaxf(db, floor_db);
}

}  // namespace

hipError_t launch_backproject(const BackProjArgs &a, hipStream_t s)
{
    if (a.n_vox <= 0) return hipSuccess;
    if (a.K < 1 || a.K > RR_BP_KMAX) return hipErrorInvalidValue;
    const int64_t blocks = (a.n_vox + BP_T - 1) / BP_T;
    hipLaunchKernelGGL(k_backproject, dim3((unsigned)blocks), dim3(BP_T), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_max_projection(const float2 *img, int64_t nx, int64_t nyz, float *out,
                                 float *peak, float floor_db, hipStream_t s)
{
    if (nyz <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((nyz + 255) / 256);
    hipLaunchKernelGGL(k_max_projection, dim3(blocks), dim3(256), 0, s, img, nx, nyz, out, peak);
    hipLaunchKernelGGL(k_to_db, dim3(blocks), dim3(256), 0, s, out, nyz, peak, floor_db);
    return hipGetLastError();
}
