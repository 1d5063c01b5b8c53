// Internal declarations shared by the host code and the kernel launchers of
// libradray.  Not part of the public ABI (see include/radray.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/radray.h"

#define RR_TRACE_BLOCK 128
#define RR_STACK 32          // BVH depth bound (the builder guarantees depth <= 31)
#define RR_LEAF_MAX 8        // triangles per leaf (3-bit count in the child reference)

// ---------------------------------------------------------------------------
// device-side structure-of-arrays path list (planes of `cap` elements)
// ---------------------------------------------------------------------------
struct PathSoA {
    int32_t *src = nullptr;
    int32_t *K = nullptr;
    int64_t *ray = nullptr;
    int32_t *loc = nullptr;   // index of the path among its ray's paths (temp list only)
    int32_t *tri = nullptr;   // [RR_KMAX][cap]
    int32_t *vid = nullptr;   // [RR_KMAX][cap]
    double *p = nullptr;      // [RR_KMAX*3][cap]
    double *L = nullptr;
    double *amp = nullptr;
    int64_t cap = 0;
};

// ---------------------------------------------------------------------------
// BVH on the device.  Node (64 B): child boxes and child references
//   n[0] = (lo0.x, lo0.y, lo0.z, hi0.x)   n[1] = (hi0.y, hi0.z, lo1.x, lo1.y)
//   n[2] = (lo1.z, hi1.x, hi1.y, hi1.z)   n[3] = (ref0, ref1, 0, 0) as int bits
// Reference r >= 0: internal node r.  r < 0: leaf, x = ~r, first triangle
// x >> 3 of the leaf-ordered triangle array, count (x & 7) + 1.
// Leaf triangle (48 B): (v0.xyz, v1.x) (v1.yz, v2.xy) (v2.z, id, obj, 0)
// with id/obj stored as int bits.
// ---------------------------------------------------------------------------
struct HostBvh {
    std::vector<float> nodes;    // 16 floats per node
    std::vector<float> tris;     // 12 floats per triangle
    int depth = 0;
};

// Field of view of a per-triangle launch as seen from its sources (the Tx
// phase centre, or every Tx element): cosines and sines of the azimuth
// bounds, sines of the elevation bounds.
struct RrFov {
    const double *src;
    int32_t n_src;
    double c0, s0, c1, s1, slo, shi;
};
int rr_build_pieces(const float *verts, const int32_t *tris, int64_t n_tris, const double *o,
                    double omega_max, int depth_max, const RrFov *fov, int64_t limit,
                    std::vector<double> &pverts, std::vector<int32_t> &parent);
int rr_build_bvh(const float *verts, int64_t nv, const int32_t *tris, const int32_t *tri_obj,
                 const float *obj_alpha, int64_t nt, HostBvh &out, std::string &err);

// ---------------------------------------------------------------------------
// trace kernel arguments (by value)
// ---------------------------------------------------------------------------
struct TraceArgs {
    const float4 *nodes;
    const float4 *ltris;
    int has_bvh;
    const double *tx;         // [ntx][3]
    const double *pt_pos;     // [npts][3]
    const double *pt_ap;      // [npts]
    double oT[3], oR[3];
    double r2;
    int shared;
    int nobj, npts;
    int64_t n_src, n_per_src, n_virt_per_src;
    double at, bt, slo, shi, omega;
    int bmax;
    uint64_t seed;
    int sampler;
    const double *cdf;
    int n_az, n_el;
    const double *pieces;     // [n_pieces][9] vertices of the per-triangle launch's pieces
    const int32_t *piece_parent;   // [n_pieces] triangle a piece's rays must hit first
    int tri_g;                // g: g^2 rays per piece and source
    double fov_c0, fov_s0, fov_c1, fov_s1;   // cos, sin of the azimuth bounds
    int64_t vbase;            // first virtual ray of this scene in the (batched) ray space
    const int32_t *order;     // [n_traced] ray of each lane (coherent order) or null
    // outputs
    int32_t *hits;            // [n_src*n_per_src][bmax+1] or null
    uint8_t *counts;          // indexed by vbase + virtual ray
    PathSoA tmp;
    unsigned long long *counter;
    int *err_flag;
};

// caller-supplied rays (device arrays)
struct UserRays {
    const double *orig;       // [n][3]
    const double *dir;        // [n][3]
    const double *amp;        // [n]
    const int32_t *src;       // [n]
    int64_t n;
};

// ---------------------------------------------------------------------------
// synthesis path record (AoS, prepared from the path list)
// ---------------------------------------------------------------------------
struct SynPath {
    double P[RR_KMAX][3];     // hit points at t = 0
    double V[RR_KMAX][3];     // their velocities
    double amp;
    int32_t K;
    int32_t src;
};

struct SynthArgs {
    const SynPath *paths;
    const int64_t *ranges;    // [n_groups + 1] path range of each group
    int64_t n_paths;
    const double *tx, *rx;    // device [n][3]
    int ntx, nrx;
    double oT[3], oR[3];
    int shared;
    int model;
    double f0, bw, t_rep, inv_c;
    int M, K;
    float2 *cube;
    int64_t p_limit;          // > 0: at most this many paths of each group (tile timing only)
};

// back-projection (imaging): one single-sweep cube onto a voxel grid
#define RR_BP_KMAX 4096          // longest sweep: one channel fills the staging buffer
struct BackProjArgs {
    const float2 *cube;       // channel c's sweep at cube + c * stride
    int64_t stride;
    const double *tx, *rx;    // device [n][3]
    int ntx, nrx, C, K;
    double f0, df, inv_c;
    double x0, y0, z0, step;  // voxel (i, j, k) at (x0 + i step, y0 + j step, z0 + k step)
    int nx, ny, nz;
    int64_t n_vox;
    float2 *image;            // [nx][ny][nz]
};

// largest samples-per-lane tile of the batched synthesis kernel (its
// register use, hence its occupancy, follows the largest tile it contains)
#ifndef RR_BATCH_MAX_KR
#define RR_BATCH_MAX_KR 32
#endif

// batched launch: per-scene tables read by the persistent kernels
struct BatchSynthInfo {
    int kr;                   // samples per lane (tile shape)
    int rows_per_group;
    int rc;                   // channels per group
    int bpg;                  // workgroups per group
};
struct BatchVel {
    const double *obj_vel;
    const double *pt_vel;
    int nobj, npts;
};
struct BatchRangeInfo {
    int64_t vr0;              // first virtual ray of the scene
    int64_t n_vps;            // virtual rays per source
    int64_t base;             // first entry of the scene in the ranges table
    int n_groups;
    int shared;
};

// launchers (defined in the .hip files)
hipError_t launch_trace(const TraceArgs &a, int64_t n_traced, hipStream_t s);
// coherent ray order of a uniform or proposal launch: rays sorted by source
// and the 2^bits x 2^bits cell of their first direction (cells: n_src 4^bits
// counters, ray_cells: n_traced cell numbers, order: n_traced ray indices)
int trace_order_bits(int64_t n_per_src);
hipError_t launch_trace_order(const TraceArgs &a, int64_t n_traced, int bits, unsigned *cells,
                              uint16_t *ray_cells, int32_t *order, hipStream_t s);
hipError_t launch_points(const TraceArgs &a, hipStream_t s);
// k_trace plus exact work counters: stats[0] BVH nodes fetched, stats[1] leaf
// triangle records fetched, stats[2] closest-hit queries (summed, not cleared)
hipError_t launch_trace_count(const TraceArgs &a, int64_t n_traced, unsigned long long *stats,
                              hipStream_t s);
hipError_t launch_trace_user(const TraceArgs &a, const UserRays &u, hipStream_t s);
hipError_t launch_set_alpha(float4 *ltris, int64_t n_tris, const float *tri_alpha,
                            const float *obj_alpha, hipStream_t s);
hipError_t launch_bp_mfma(const float2 *cube, int64_t stride, const double *tx, int T,
                          const double *rx, int R, int K, double f0, double df, double inv_c,
                          double x0, double y0, double z0, double step, int nx, int ny, int nz,
                          uint4 *Sf, float2 *image, hipStream_t s);
int64_t bp_mfma_frag_bytes(int K);
int freq_k_step();
int freq_k_group();   // samples per exact-GEMM workgroup
// leg tables of n paths, or (rng_lo != NULL) of the records *rng_lo ..
// *rng_hi of `paths` read on the device, at most Ppad of them; own_tx: one X
// row per chirp, each path's own transmitter (see freq_own_tx)
hipError_t launch_freq_prep(const SynPath *paths, int64_t n, const int64_t *rng_lo,
                            const int64_t *rng_hi, int64_t Ppad, int M, double t_rep,
                            const double *tx, int T, bool own_tx, const double *rx, int R,
                            double f0c, double dfc, uint2 *xt, uint2 *yt, float *amp, int32_t *src,
                            hipStream_t s);
// the X table keeps one row per chirp (each path's own transmitter) for a
// per-element launch on the sample split with transmitter groups, else one
// per (chirp, transmitter); entries (8 bytes each) of both tables
bool freq_own_tx(int tile, bool per_element, bool has_groups);
int64_t freq_table_entries(int T, int R, int M, int64_t Ppad, bool own_tx);
// exact product engine layouts: Tx x Rx tile 16, 32, 48, 64 or 96, or 1 (one
// channel per wavefront, samples split); the layout of least modelled time,
// the modelled time (relative) of one, and the path splits of a launch
int freq_tile(int T, int R, int K, bool per_element);
double freq_tile_cost(int T, int R, int K, int tile, bool per_element);
void freq_splits(int tile, int T, int R, int M, int K, int64_t Ppad, int &n_split, int64_t &split_len);
// the exact model's AUTO rule: the best product layout is modelled at least
// 1.5x the direct engine's throughput
bool freq_pays(int T, int R, int K, bool per_element);
// rng_lo / rng_hi (may be NULL): the path count read on the device, as for
// launch_freq_prep; the splits then divide that count evenly.  groups (may be
// NULL; per-element launch, tile 1): [T + 1] path range of each transmitter
// in the list the tables were built from (offset by groups[0])
hipError_t launch_freq_gemm(const uint2 *xt, const uint2 *yt, const float *amp, const int32_t *src,
                            int T, int R, int M, int K, int64_t Ppad, int n_split, int64_t split_len,
                            int per_element, int tile, const int64_t *rng_lo, const int64_t *rng_hi,
                            const int64_t *groups, float2 *partial, float2 *cube, hipStream_t s);
hipError_t launch_refit(float4 *nodes, float *ubox, const int32_t *order,
                        const int64_t *level_start, int n_levels, float4 *ltris, int64_t n_tris,
                        const int32_t *tris, const float *verts, double pad, hipStream_t s);
hipError_t launch_backproject(const BackProjArgs &a, hipStream_t s);
hipError_t launch_max_projection(const float2 *img, int64_t nx, int64_t nyz, float *out,
                                 float *peak, float floor_db, hipStream_t s);
hipError_t launch_check_user(const UserRays &u, int shared, int ntx, int *flag, hipStream_t s);
hipError_t launch_scan_u8(const uint8_t *counts, int64_t n, uint32_t *offsets, uint32_t *bsums,
                          int64_t nb_cap, unsigned long long *total, hipStream_t s);
int64_t scan_u8_blocks(int64_t n);
hipError_t launch_scatter(const PathSoA &tmp, const unsigned long long *counter, int64_t tmp_cap,
                          const uint32_t *offsets, const PathSoA &dst, int64_t keep,
                          hipStream_t s);

hipError_t launch_syn_prep(const PathSoA &paths, int64_t n, const double *obj_vel, int nobj,
                           const double *pt_vel, int npts, SynPath *out, hipStream_t s);
hipError_t launch_ranges(const int32_t *src, int64_t n, int n_groups, int g0, int64_t *ranges,
                         hipStream_t s);
hipError_t launch_synth_direct(const SynthArgs &a, int n_groups, int rows_per_group,
                               hipStream_t s);
hipError_t launch_synth_sampled(const SynthArgs &a, const int64_t *idx, int64_t n_idx,
                                hipStream_t s);

// split-bf16 complex GEMM engine (k_gemm.hip)
int gemm_row_pad();
int gemm_a_bytes();
int gemm_col_tile();
int gemm_k_step();
hipError_t launch_gemm_prep_tr(const SynthArgs &a, int Ppad, float2 *T, float2 *R, hipStream_t s);
hipError_t launch_gemm_prep_a(const float2 *T, const float2 *R, int nrx, int C, int Cpad, int Ppad,
                              uint4 *Af, hipStream_t s);
hipError_t launch_gemm_prep_b(const SynthArgs &a, int Ppad, uint4 *Bp, hipStream_t s);
hipError_t launch_gemm_main(const uint4 *Af, const uint4 *Bp, int Cpad, int Ppad, int C, int M,
                            int K, float2 *cube, hipStream_t s);

// learned proposal (k_trace.hip: probe and histogram; k_mlp.hip: network)
hipError_t launch_probe(const TraceArgs &a, float *code, hipStream_t s);
hipError_t launch_hist(const TraceArgs &a, int64_t n_traced, const int32_t *hits,
                       const int32_t *tri_obj, int n_az, int n_el, float *H, hipStream_t s);
#include <hip/hip_fp16.h>
hipError_t launch_mlp_forward(const float *P, const float *codes, int64_t n, __half *acts, float *z,
                              hipStream_t s);
hipError_t launch_softmax_grad(const float *z, const float *H, int n_scenes, float *dz, float *loss,
                               hipStream_t s);
// weight gradients: the rows are split over at most 4 096 blocks, each
// writing its partial sums into part; two passes then add them in a fixed
// order (runs of consecutive blocks, then the runs) into grad (every entry
// written).  part holds mlp_part_rows(n) rows of RR_MLP_PARAMS floats.
int64_t mlp_part_rows(int64_t n);
hipError_t launch_mlp_backward(const float *P, const float *dz, int64_t n, const __half *acts,
                               float *d1, float *d2, float *d3, const float *codes, float *part,
                               float *grad, hipStream_t s);
hipError_t launch_adam(float *P, const float *G, float *m, float *v, float lr, int step, hipStream_t s);
hipError_t launch_build_cdf(const float *z, float beta, float power, float kappa, double *cdf,
                            hipStream_t s);
hipError_t launch_batch_trace(const TraceArgs *scenes, const int64_t *chunk_start, int S,
                              int64_t n_chunks, unsigned long long *work, hipStream_t s);
hipError_t launch_batch_synth(const SynthArgs *scenes, const BatchSynthInfo *info,
                              const int64_t *item_start, int S, int64_t n_items,
                              unsigned long long *work, hipStream_t s);
hipError_t launch_batch_prep(const PathSoA &paths, const unsigned long long *total, int64_t cap,
                             const int64_t *vr_start, int S, const BatchVel *vel, SynPath *out,
                             hipStream_t s);
hipError_t launch_batch_ranges(const uint32_t *offsets, int64_t V, const unsigned long long *total,
                               int64_t cap, const BatchRangeInfo *ri, int S, int64_t *ranges,
                               hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
