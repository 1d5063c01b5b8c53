// k_refit.hip -- refit of the tracer's BVH to moved vertices (same topology):
// animated or deforming meshes (hand movements) traced frame by frame
// without a host rebuild.
//
// Leaf records (12 words: 9 vertex coordinates, upload index, object, alpha)
// take the new vertex positions; then the tree is refit bottom-up, one launch
// per depth, deepest first.  For every node the exact FP32 bounds of each
// child's subtree (a leaf's triangles, or the child node's own exact bounds,
// kept in a side array) are padded and rounded outward exactly as the host
// build pads them, so an unchanged mesh refits to the identical tree and a
// moved mesh gets boxes that can only over-include.
#include <cfloat>

#include "rr_internal.h"

namespace {

__global__ void k_refit_leaves(float *ltris, int64_t nt, const int32_t *tris, const float *verts)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    float *T = ltris + 12 * k;
    const int id = __float_as_int(T[9]);
    for (int c = 0; c < 3; c++) {
        const int64_t vi = tris[3 * (int64_t)id + c];
        for (int a = 0; a < 3; a++) T[3 * c + a] = verts[3 * vi + a];
    }
}

// FP32 box padded by pad (in FP64) and rounded outward, as the host build
__device__ __forceinline__ void padded(const float *lo, const float *hi, double pad, float *out)
{
    for (int a = 0; a < 3; a++) {
        float l = (float)((double)lo[a] - pad);
        if ((double)l > (double)lo[a] - pad) l = nextafterf(l, -FLT_MAX);
        float h = (float)((double)hi[a] + pad);
        if ((double)h < (double)hi[a] + pad) h = nextafterf(h, FLT_MAX);
        out[a] = l;
        out[3 + a] = h;
    }
}

__global__ void k_refit_level(float *nodes, float *ubox, const int32_t *order, int64_t n,
                              const float *ltris, double pad)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t node = order[k];
    float *N = nodes + 16 * (int64_t)node;
    const int32_t ref0 = __float_as_int(N[12]), ref1 = __float_as_int(N[13]);
    float lo[2][3], hi[2][3];
    for (int c = 0; c < 2; c++) {
        const int32_t ref = c ? ref1 : ref0;
        for (int a = 0; a < 3; a++) {
            lo[c][a] = FLT_MAX;
            hi[c][a] = -FLT_MAX;
        }
        if (ref < 0) {
            const int32_t code = ~ref;
            const int64_t first = code >> 3, count = (code & 7) + 1;
            for (int64_t q = first; q < first + count; q++) {
                const float *T = ltris + 12 * q;
                for (int v = 0; v < 3; v++)
                    for (int a = 0; a < 3; a++) {
                        lo[c][a] = fminf(lo[c][a], T[3 * v + a]);
                        hi[c][a] = fmaxf(hi[c][a], T[3 * v + a]);
                    }
            }
        } else {
            const float *U = ubox + 6 * (int64_t)ref;
            for (int a = 0; a < 3; a++) {
                lo[c][a] = U[a];
                hi[c][a] = U[3 + a];
            }
        }
    }
    float *U = ubox + 6 * (int64_t)node;
    for (int a = 0; a < 3; a++) {
        U[a] = fminf(lo[0][a], lo[1][a]);
        U[3 + a] = fmaxf(hi[0][a], hi[1][a]);
    }
    float b[6];
    padded(lo[0], hi[0], pad, b);
    for (int q = 0; q < 6; q++) N[q] = b[q];
    // a root that is a single leaf holds it twice, the second copy behind a
    // box far outside the scene: keep that box
    if (ref1 != ref0 || ref0 >= 0) {
        padded(lo[1], hi[1], pad, b);
        for (int q = 0; q < 6; q++) N[6 + q] = b[q];
    }
}

}  // namespace

hipError_t launch_refit(float4 *nodes, float *ubox, const int32_t *order,
                        const int64_t *level_start, int n_levels, float4 *ltris, int64_t n_tris,
                        const int32_t *tris, const float *verts, double pad, hipStream_t s)
{
    if (n_tris <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refit_leaves, dim3((unsigned)((n_tris + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<float *>(ltris), n_tris, tris, verts);
    // levels are stored deepest first: level_start[l] .. level_start[l + 1]
    for (int l = 0; l < n_levels; l++) {
        const int64_t a = level_start[l], n = level_start[l + 1] - a;
        if (n <= 0) continue;
        hipLaunchKernelGGL(k_refit_level, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s,
                           reinterpret_cast<float *>(nodes), ubox, order + a, n,
                           reinterpret_cast<const float *>(ltris), pad);
    }
    return hipGetLastError();
}
