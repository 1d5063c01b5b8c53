/*
 * radray.h -- C ABI of the MI355X radar ray-tracing library (libradray.so).
 *
 * The library computes the hot path of the ray-tracing radar simulator of
 * Braeunig et al., "A Realistic Radar Ray Tracing Simulator for Hand Pose
 * Imaging" (Section III): rays leave every transmitter, bounce off a
 * triangle mesh with the two-lobe material of Eqs. (1)-(3), the received
 * paths keep their total length (Section III-B), and the baseband is the
 * coherent sum of Eq. (4).  Eq. (4) is evaluated with the FMCW instantaneous
 * frequency f_k = f0 + B k / K of fast-time sample k instead of the stepped
 * frequency, and objects move at constant velocity between chirps
 * (stop-and-go).  All device work runs in hand-written HIP kernels for gfx950.
 *
 * Conventions shared by every entry point
 *   - Return value: RR_OK (0) or a negative RR_E* code; no exception crosses
 *     the ABI.  rr_last_error() returns a thread-local message for the last
 *     failing call on the calling thread.
 *   - Units: metres, seconds, hertz.  Axes: x = boresight, y = left, z = up.
 *   - Host pointers (`const T*` without `_dev`) are read during the call and
 *     copied; the caller keeps ownership.  Device pointers (`*_dev`) are
 *     caller-owned HIP allocations on the context's device; they must stay
 *     valid until the work enqueued by the call has completed on the
 *     context's stream.
 *   - All device work is enqueued on the stream given to rr_create, in call
 *     order.  A call returns without waiting unless it writes a host scalar
 *     (`*_out` arguments), which synchronises the stream.
 *   - Virtual channel c = t * n_rx + r (Tx-major).  Cubes are complex64
 *     (interleaved float re, im) laid out [channel][chirp][sample].
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef RADRAY_H
#define RADRAY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RR_OK = 0,
    RR_EINVAL = -1,        /* invalid argument (shape, NaN, range) */
    RR_ENOMEM = -2,        /* device or host allocation failed */
    RR_EHIP = -3,          /* a HIP runtime call failed */
    RR_ESTATE = -4,        /* call order violated (e.g. synthesize before trace) */
    RR_EOVERFLOW = -5,     /* an output buffer is too small; needed size reported */
    RR_EUNSUPPORTED = -6   /* valid request that this library does not support */
};

enum { RR_TX_PER_ELEMENT = 0, RR_TX_SHARED = 1 };
enum { RR_UNIFORM = 0, RR_PROPOSAL = 1, RR_PER_TRIANGLE = 2 };
enum { RR_EXACT = 0, RR_SEPARABLE = 1 };
enum { RR_ENGINE_AUTO = 0, RR_DIRECT_FP32 = 1, RR_GEMM_BF16X3 = 2, RR_GEMM_EXACT = 3 };

#define RR_KMAX 4          /* largest supported bounce count */

typedef struct rr_ctx rr_ctx;

/* Create a context on HIP device `hip_device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
int rr_create(int hip_device, void *hip_stream, rr_ctx **out);

/* Release every device buffer the context owns.  Safe on NULL. */
void rr_destroy(rr_ctx *ctx);

/* Message of the last failing call on this thread ("" if none). */
const char *rr_last_error(void);

/* Library version string. */
const char *rr_version(void);

/* Scene upload (Section III: a 3D triangle mesh; Sec. III-A: a material
 * parameter alpha per surface, Eq. 3).
 *   verts     float [n_verts][3]
 *   tris      int32 [n_tris][3] vertex indices
 *   tri_obj   int32 [n_tris] object of each triangle, in [0, n_obj)
 *   obj_alpha float [n_obj], each in [0, 1] (0 specular, 1 diffuse)
 *   obj_vel   double [n_obj][3] constant velocity (m/s)
 *   pt_pos, pt_vel double [n_pts][3], pt_aperture double [n_pts] (m^2):
 *             point reflectors (a retro-reflector of the given aperture)
 * The host builds a binned-SAH BVH (depth <= 31) and uploads it.  Replaces
 * any previous scene and invalidates traced paths.  n_tris may be 0.
 * Errors: RR_EINVAL for out-of-range indices, non-finite coordinates or alpha
 * outside [0, 1]; RR_ENOMEM. */
int rr_scene_upload(rr_ctx *ctx, const float *verts, int64_t n_verts,
                    const int32_t *tris, const int32_t *tri_obj, int64_t n_tris,
                    const float *obj_alpha, const double *obj_vel, int32_t n_obj,
                    const double *pt_pos, const double *pt_vel, const double *pt_aperture,
                    int32_t n_pts);

/* Move the uploaded scene's vertices (same count, same triangles): for
 * animated or deforming meshes such as moving hands (Sec. V), traced frame
 * by frame.  verts float [n_verts][3], host, copied.  Instead of a host
 * rebuild the BVH is refit on the GPU: leaf triangles take the new
 * positions, then every node's child boxes are recomputed bottom-up (one
 * launch per depth) from the exact bounds of the child subtrees, padded and
 * rounded outward like the host build, so traversal stays exact (boxes only
 * over-include); an unchanged mesh refits to the identical tree.  The
 * topology of the tree is kept, so large motions can make traversal slower,
 * never wrong.  Drains the context's stream first; later traces see the new
 * geometry, paths already traced are kept.
 * Errors: RR_ESTATE (no scene), RR_EINVAL (count differs from the upload,
 * NULL or non-finite vertices). */
int rr_scene_update_vertices(rr_ctx *ctx, const float *verts, int64_t n_verts);

/* Copy of the BVH node array (16 floats per node: both child boxes, lo.xyz
 * hi.xyz each, then the two child references as int32 bits: >= 0 a node,
 * < 0 the leaf ~(first << 3 | (count - 1)) of leaf-ordered triangles) for
 * inspection.  dst host (NULL: only *n_floats is written); capacity in
 * floats.  Errors: RR_ESTATE, RR_EOVERFLOW (capacity too small). */
int rr_get_bvh_nodes(rr_ctx *ctx, float *dst, int64_t capacity, int64_t *n_floats);

enum { RR_ALPHA_PER_OBJECT = 0, RR_ALPHA_PER_TRIANGLE = 1 };

/* Replace the material mix alpha of Eq. 3 (Sec. III-A) of the uploaded scene
 * without rebuilding the BVH: for a sweep of alpha over one mesh (the paper
 * varies alpha from 0 to 1 in steps of 0.1, Sec. IV) and per-face variation
 * for data diversity (Sec. V).
 *   alpha float [n], host, copied; each in [0, 1].
 *   per   RR_ALPHA_PER_OBJECT: n = n_obj, every face takes its object's value;
 *         RR_ALPHA_PER_TRIANGLE: n = n_tris, face i (upload index) takes
 *         alpha[i], overriding its object's.
 * Drains the context's stream, then enqueues the update on it; traces issued
 * later see the new values, earlier traced paths are kept.
 * Errors: RR_ESTATE without a scene; RR_EINVAL for a wrong count, an unknown
 * mode or a value outside [0, 1] (nothing is changed then). */
int rr_scene_set_alpha(rr_ctx *ctx, const float *alpha, int64_t n, int32_t per);

/* MIMO array geometry (Section II).  tx double [n_tx][3], rx double [n_rx][3].
 * rx_radius: radius of the array-level reception sphere centred on the Rx
 * phase centre (mean of rx).  tx_mode: RR_TX_PER_ELEMENT (rays from every Tx,
 * n_rays / n_tx each) or RR_TX_SHARED (rays from the Tx phase centre, each
 * path feeding every channel).  Errors: RR_EINVAL. */
int rr_set_array(rr_ctx *ctx, const double *tx, int32_t n_tx, const double *rx, int32_t n_rx,
                 double rx_radius, int32_t tx_mode);

/* FMCW chirp: start frequency f0, sweep bandwidth B over t_chirp, chirp
 * repetition t_rep, n_samples fast-time samples per chirp (sample k at
 * frequency f0 + B k / n_samples), n_chirps chirps.  Errors: RR_EINVAL. */
typedef struct {
    double f0, bandwidth, t_chirp, t_rep;
    int32_t n_samples, n_chirps;
} rr_chirp;
int rr_set_chirp(rr_ctx *ctx, const rr_chirp *chirp);

/* Trace parameters (Sec. III-A: each Tx sends out many rays).
 *   n_rays      total launched rays (split evenly over Tx in per-element mode);
 *               with RR_PER_TRIANGLE: rays cast towards each triangle from
 *               each source, a perfect square g^2 >= 1
 *   max_bounces surface hits per ray, 1..RR_KMAX
 *   seed        Philox4x64-10 key
 *   az/el range field of view in radians; directions uniform in solid angle
 *   sampler     RR_UNIFORM, or RR_PROPOSAL (bins of the proposal table set by
 *               rr_proposal_set_cdf or rr_proposal_build, weight p0/q), or
 *               RR_PER_TRIANGLE (Sec. III: rays cast towards every mesh
 *               triangle): each triangle is first cut into pieces, and
 *               pieces out of view are dropped (see rr_set_casting; by
 *               default the pieces are the triangles in view);
 *               ray k of piece f (virtual ray f g^2 + k of its source) aims at
 *               a point uniform in cell (k mod g, k / g) of a g x g grid,
 *               mapped area-preservingly onto the piece, with weight
 *               p0 A |cos theta| / d^2 / g^2 (A the piece's area, p0 = 1 /
 *               field-of-view solid angle): the same estimate as the uniform
 *               launch.  Rays outside the field of view, and rays whose first
 *               hit is not the piece's parent triangle, are not counted (hit
 *               row all -1).  Needs an azimuth span of at most pi.
 *   record_hits 1: keep the per-ray hit list for rr_get_hits
 *   path_cap    keep at most this many paths (first in ray, bounce order);
 *               0 = keep all */
typedef struct {
    int64_t n_rays;
    int32_t max_bounces;
    uint64_t seed;
    double az_min, az_max, el_min, el_max;
    int32_t sampler;
    int32_t record_hits;
    int64_t path_cap;
} rr_trace_params;

/* Trace the scene from the array.  Paths are ordered by (virtual ray,
 * bounce): for source s, its rays 0..N_s-1 then its point reflectors.  With
 * n_paths_out != NULL the stream is synchronised and the number of stored
 * paths written; the internal path buffer grows as needed.  With NULL the
 * call does not synchronise: the path count stays on the device until a call
 * that needs it on the host (rr_get_path_count, rr_get_paths, rr_get_hits,
 * rr_synthesize, rr_proposal_histogram) reads it back with one
 * synchronisation; if the paths overflowed the current temporary buffer, that
 * call returns RR_EOVERFLOW, the buffer grows and the trace must be repeated.
 * Uniform and proposal launches of at least 4096 rays per source trace their
 * rays in a coherent order (sorted by source and first-direction cell, which
 * costs n_rays x 6 bytes of device memory); hits, counts and paths are the
 * same as in ray order, bit for bit.
 * Errors: RR_ESTATE (no scene or array), RR_EINVAL, RR_ENOMEM, RR_EHIP,
 * RR_EUNSUPPORTED (a BVH deeper than the traversal stack; the builder keeps
 * depth <= 31, so this is not expected). */
int rr_trace(rr_ctx *ctx, const rr_trace_params *params, int64_t *n_paths_out);

/* rr_trace run by a variant of the tracing kernel that also counts its work
 * (the same hits and paths bit for bit, somewhat slower): the data behind the
 * tracer's memory roofline (Sec. IV: the tracer's cost grows with the mesh).
 * work_out[0] rays traced (point reflectors excluded), [1] closest-hit
 * queries (segments), [2] BVH nodes fetched (64 B each), [3] leaf triangle
 * records fetched (48 B each).  n_paths_out is required (the call
 * synchronises).  Errors as rr_trace. */
int rr_trace_work(rr_ctx *ctx, const rr_trace_params *params, int64_t *n_paths_out,
                  int64_t work_out[4]);

/* Pieces of the RR_PER_TRIANGLE launch (Sec. III casts rays towards every
 * triangle; a coarse mesh with a large near triangle gets its rays spread by
 * cutting it).  Every triangle, in upload order, is cut by midpoint
 * subdivision into four while the piece subtends more than max_solid_angle
 * steradians from the Tx phase centre (Van Oosterom-Strackee formula, FP64)
 * and its depth is below max_depth; the children of (a, b, c) are
 * (a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca), depth first.
 * Pieces none of whose rays can enter the trace's field of view are dropped:
 * all three vertices beyond the same bounding plane of the azimuth wedge, or
 * inside the same excluded elevation cone where that cone is convex (below
 * el_min <= 0, above el_max >= 0), by a margin of 1e-9 of their distance, as
 * seen from every source (the Tx phase centre, or each Tx element).
 * max_solid_angle = 0 (the default, with max_depth 8) casts at the triangles
 * in view.  Takes effect at the next per-triangle trace; the pieces are
 * rebuilt on the host after a change of these parameters, the field of view,
 * the scene, its vertices or the array.  Errors: RR_EINVAL (negative or
 * non-finite angle, max_depth outside [0, 20]). */
int rr_set_casting(rr_ctx *ctx, double max_solid_angle, int32_t max_depth);

/* Number of pieces a RR_PER_TRIANGLE trace with the field of view of params
 * casts at (only az/el of params are read; builds the pieces if needed); such
 * a trace launches n_pieces * n_rays rays per source.  Errors: RR_ESTATE (no
 * scene or array), RR_EOVERFLOW (more than 2^26 pieces), RR_EINVAL (NULL, or
 * a field of view per-triangle casting does not take). */
int rr_casting_pieces(rr_ctx *ctx, const rr_trace_params *params, int64_t *n_pieces);

/* Trace caller-supplied rays instead of the launch (Sec. III-A sends rays
 * out from each transmitter; here the caller chooses them, e.g. for another
 * launch density or rays cast at given triangles).
 *   orig_dev, dir_dev double [n][3]: origin and direction of ray i (the
 *                     direction is normalised here; it must be non-zero)
 *   amp_dev  double [n]: amplitude of every path ray i produces (the launch
 *                     uses w / N_t)
 *   src_dev  int32 [n]: -1 for every ray with a RR_TX_SHARED array; with
 *                     RR_TX_PER_ELEMENT the Tx index in [0, n_tx), ascending
 *                     over i (each path feeds its Tx's channels)
 * Bounces, reception and path bookkeeping are those of rr_trace, with the
 * random numbers of the bounce at hit j drawn from counter (i - i0, src, j + 1)
 * (i0: the first ray of the same source, src: 0 for -1), so that the launch's
 * own rays reproduce rr_trace exactly.  Point reflectors are not traced.
 * Paths are ordered by (ray, bounce) with ray = i; with record_hits the hit
 * list has n rows (rr_get_hits).  Synchronises; n_paths_out may be NULL.
 * Errors: RR_ESTATE (no scene or array), RR_EINVAL (bad bounce count, NULL
 * arrays, a source out of range or not ascending, a non-finite value or a
 * zero direction, found by a device check before tracing), RR_ENOMEM. */
int rr_trace_rays(rr_ctx *ctx, const double *orig_dev, const double *dir_dev,
                  const double *amp_dev, const int32_t *src_dev, int64_t n,
                  int32_t max_bounces, uint64_t seed, int32_t record_hits, int64_t *n_paths_out);

/* Number of paths held by the context (synchronises).  RR_EOVERFLOW (with
 * the needed count in *n_out) if the last asynchronous trace overflowed. */
int rr_get_path_count(rr_ctx *ctx, int64_t *n_out);

/* Copy the per-ray hit list of the last trace into tri_dev, int32
 * [n_rays][max_bounces + 1]: closest-hit triangle id of each traced segment,
 * -1 for a miss or a segment not traced.  Ray r of source s is row
 * s * N_s + r.  cap_elems is the capacity of tri_dev in elements.
 * Errors: RR_ESTATE (no hits recorded), RR_EOVERFLOW. */
int rr_get_hits(rr_ctx *ctx, int32_t *tri_dev, int64_t cap_elems);

/* Path list in structure-of-arrays form (device pointers, planes of
 * `stride` elements):
 *   src  int32  [n]      Tx index, -1 for a shared launch
 *   K    int32  [n]      number of hit points (1..RR_KMAX)
 *   ray  int64  [n]      virtual ray id
 *   tri  int32  [RR_KMAX][stride]  hit triangle ids (-1: point reflector/unused)
 *   vid  int32  [RR_KMAX][stride]  velocity id: object id, or n_obj + point id
 *   p    double [RR_KMAX*3][stride] hit point j, coordinate a in plane 3j+a
 *   L    double [n]      source-to-last-hit length at t = 0
 *   amp  double [n]      amplitude a_p (weight / rays per source, or the
 *                        point reflector's return) */
typedef struct {
    int32_t *src;
    int32_t *K;
    int64_t *ray;
    int32_t *tri;
    int32_t *vid;
    double *p;
    double *L;
    double *amp;
    int64_t stride;
} rr_paths;

/* Copy the context's paths into dst (device buffers, capacity dst->stride).
 * *n_out receives the number of paths (synchronises).  RR_EOVERFLOW if the
 * capacity is too small (the needed count is still written to *n_out). */
int rr_get_paths(rr_ctx *ctx, const rr_paths *dst, int64_t *n_out);

/* Replace the context's paths by n paths from src (device buffers), e.g. to
 * synthesise a path list produced elsewhere.  Errors: RR_EINVAL, RR_ENOMEM. */
int rr_set_paths(rr_ctx *ctx, const rr_paths *src, int64_t n);

/* Coherent sum of Eq. (4) over the context's paths into cube_dev.
 *   model  RR_EXACT: d = |p_1(m) - tx_t| + inner(m) + |rx_r - p_K(m)| per
 *          channel and chirp; RR_SEPARABLE: the channel part of the length
 *          uses f0 and chirp 0 (a per-channel factor times a per-(chirp,
 *          sample) factor), which allows the complex-GEMM engine.
 *   engine RR_DIRECT_FP32 (either model), RR_GEMM_BF16X3 (separable only:
 *          split-bf16 hi+lo complex GEMM on MFMA, FP32 accumulation; each
 *          chirp's samples are computed in whole tiles of 64; relative error
 *          bar 1e-3), RR_GEMM_EXACT (exact model only, full cube: split-bf16
 *          complex products on the matrix cores of FP64-reduced leg phases,
 *          held to the exact model's 1e-4 bar; either one (Tx x paths) by
 *          (paths x Rx) product per (chirp, sample) in square tiles of 16,
 *          32, 48, 64 or 96, or, per (channel, chirp), one (k1 x paths) by
 *          (paths x k2) product over the samples k = k1 S + k2 (at most 1024
 *          samples); the layout of least modelled time), or
 *          RR_ENGINE_AUTO: the separable model takes RR_GEMM_BF16X3 when the
 *          64-sample tiling pads a chirp by at most a quarter; the exact model
 *          takes RR_GEMM_EXACT when its best layout is modelled at 1.5x
 *          the direct engine's throughput or more (in a per-element launch
 *          a path feeds only its own transmitter's channels: the Tx x Rx
 *          tiles are modelled at the work they waste, the sample split
 *          reads each transmitter's paths only) and its leg tables (8 bytes
 *          per chirp, path and element; per-element sample split: the
 *          path's own transmitter and every receiver) fit 16 GiB;
 *          everything else, and sampled entries, the direct engine.  AUTO never changes the model, and each engine
 *          it picks meets that model's error bar.
 *   cube_dev complex64 [n_ch][n_chirps][n_samples], cube_elems = its complex
 *          element count; the cube is overwritten.
 *   sample_idx_dev int64 [n_sample] flat entry indices (c*M*K + m*K + k):
 *          when non-NULL only these entries are computed, into
 *          cube_dev[0..n_sample) (direct engine, FP64-reduced phase).
 * Errors: RR_ESTATE (no paths/array/chirp), RR_EINVAL, RR_EUNSUPPORTED
 * (GEMM engine with the exact model or with sample_idx_dev). */
int rr_synthesize(rr_ctx *ctx, int32_t model, int32_t engine, void *cube_dev, int64_t cube_elems,
                  const int64_t *sample_idx_dev, int64_t n_sample);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the full
 * cube of rr_synthesize with the direct FP32 engine (either model), computed
 * without any hipMalloc, hipFree or allocating library call.  Its temporary
 * data (one synthesis record per path and the path range of each transmitter
 * group) live in a fixed scratch area of the library: at most
 * RR_NOALLOC_MAX_PATHS paths and RR_NOALLOC_MAX_TX transmitters (per-element
 * launch), about 13.7 MB that every GPU the library runs on holds from the
 * first rr_create on it until the process ends.  Inputs are the context's
 * paths, array, chirp and object velocities; cube_dev (caller-owned,
 * complex64 [n_ch][n_chirps][n_samples], cube_elems complex elements) is
 * overwritten.  The result equals rr_synthesize with RR_DIRECT_FP32 (same
 * kernels).  Paths whose source does not match the array's launch mode are
 * not summed (rr_synthesize rejects them).  All calls on one GPU share its
 * scratch and each call rewrites what it reads: calls on one stream are
 * ordered, calls that overlap in time on one GPU (other streams, other
 * contexts, other threads) race.  If the last trace left its path count on
 * the device, this call reads it back (one synchronisation, no allocation).
 * Errors: RR_ESTATE (no paths, array, chirp or scene), RR_EINVAL,
 * RR_EUNSUPPORTED (over either limit, or too many samples per chirp). */
#define RR_NOALLOC_MAX_PATHS 65536
#define RR_NOALLOC_MAX_TX 4096
int rr_synthesize_noalloc(rr_ctx *ctx, int32_t model, void *cube_dev, int64_t cube_elems);

/* ------------------------------------------------------------------------
 * Learned ray proposal (an importance-sampling density for the launch of
 * Sec. III-A).  Directions are binned on a grid of RR_PROP_NAZ azimuth x
 * RR_PROP_NEL sin(elevation) bins of equal solid angle over the field of
 * view (bin b = ie * RR_PROP_NAZ + ia).  A ray drawn from bin b gets the
 * weight 1 / (n_bins q_b), so the cube stays an unbiased estimate.
 * ------------------------------------------------------------------------ */
#define RR_PROP_NAZ 128
#define RR_PROP_NEL 64
#define RR_MLP_PARAMS 9601   /* 18 -> 64 -> 64 -> 64 -> 1, ReLU */

/* Set the sampling table explicitly: cdf double [n_az * n_el + 1] (host),
 * non-decreasing, cdf[0] = 0, last = 1.  Errors: RR_EINVAL. */
int rr_proposal_set_cdf(rr_ctx *ctx, const double *cdf, int32_t n_az, int32_t n_el);

/* Copy the current sampling table to host memory (cap entries available). */
int rr_proposal_get_cdf(rr_ctx *ctx, double *cdf, int64_t cap);

/* Scene code of the current scene: 16 azimuth sectors x 8 probe rays at
 * elevation 0 from the Tx phase centre over [az_min, az_max]; code16_dev[k]
 * = mean over the sector's rays of exp(-t / 10 m) for hits on objects other
 * than object 0 (the ground), 0 otherwise.  code16_dev: float [16] (device). */
int rr_proposal_probe(rr_ctx *ctx, double az_min, double az_max, float *code16_dev);

/* Training target from the last trace, which must have used the uniform
 * sampler with record_hits = 1: hist_dev float [RR_PROP_NAZ * RR_PROP_NEL]
 * (device, overwritten), per bin the sum over its rays of the number of
 * received paths + 0.1 if the first segment hit an object other than 0. */
int rr_proposal_histogram(rr_ctx *ctx, float *hist_dev);

/* Network parameters (FP32 master copy on the device; the kernels round
 * weights and activations to FP16 and accumulate in FP32).  Layout: W1[64][18],
 * b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[1][64], b4[1].
 * rr_mlp_init: He-uniform weights from `seed`, zero biases, Adam state reset. */
int rr_mlp_init(rr_ctx *ctx, uint64_t seed);
int rr_mlp_set_params(rr_ctx *ctx, const float *params, int64_t n);   /* host, resets Adam */
int rr_mlp_get_params(rr_ctx *ctx, float *params, int64_t n);         /* host */

/* Logits for every bin of n_scenes scenes: codes_dev float [n_scenes][16],
 * logits_dev float [n_scenes][RR_PROP_NAZ * RR_PROP_NEL] (device). */
int rr_mlp_forward(rr_ctx *ctx, const float *codes_dev, int32_t n_scenes, float *logits_dev);

/* One training step on n_scenes scenes: loss = mean over scenes of
 * -sum_b H_b log softmax(z)_b / sum_b H_b; backward pass and an Adam update
 * with learning rate lr (lr = 0: gradient only).  loss_out (host, may be
 * NULL) synchronises; grad_dev (may be NULL) receives the gradient, float
 * [RR_MLP_PARAMS]. */
int rr_mlp_train_step(rr_ctx *ctx, const float *codes_dev, const float *hist_dev, int32_t n_scenes,
                      float lr, float *loss_out, float *grad_dev);

/* `steps` Adam steps on minibatches of `batch` scenes (all scenes when
 * batch >= n_scenes), each drawn without replacement by a partial
 * Fisher-Yates shuffle driven by SplitMix64 (Steele et al. 2014) from `seed`;
 * every step is rr_mlp_train_step on the gathered rows.  codes_dev float
 * [n_scenes][16], hist_dev float [n_scenes][RR_PROP_NAZ * RR_PROP_NEL]
 * (device).  loss_out (host float [steps], may be NULL): each step's loss
 * summed over its scenes.  Synchronises only when loss_out is given.
 * Errors: RR_ESTATE (network not initialised), RR_EINVAL. */
int rr_proposal_train(rr_ctx *ctx, const float *codes_dev, const float *hist_dev, int32_t n_scenes,
                      int32_t steps, int32_t batch, float lr, uint64_t seed, float *loss_out);

/* Build the sampling table of one scene from the network: q = (1 - beta)
 * softmax(power z) + beta / n_bins, CDF in FP64.  The network is trained
 * towards the returned power per bin; power = 1 samples proportionally to it,
 * power = 1/2 proportionally to its square root, the density of least cube
 * variance for a given number of rays when every return carries the same
 * weight (importance sampling: q proportional to the root second moment of
 * a bin).  code16_dev: that scene's code (device).  Afterwards rr_trace with
 * sampler RR_PROPOSAL draws from it.  Errors: RR_ESTATE (no network),
 * RR_EINVAL (beta outside [0, 1], power outside (0, 2]). */
int rr_proposal_build(rr_ctx *ctx, const float *code16_dev, float beta, float power);

/* The sampling table of least cube variance per unit of work when both rays
 * and returned paths cost time (importance sampling: the variance goes as
 * sum_b m_b / q_b, the work as N (c_ray + c_path sum_b q_b rho_b); with every
 * return carrying about the same weight, m_b ~ rho_b, and Cauchy-Schwarz gives
 * q_b ~ sqrt(rho_b / (c_ray + c_path rho_b))).  The network's softmax is read
 * as the returns density: x_b = n_bins softmax(z)_b (1 on average), and
 *     q_b ~ sqrt(x_b / (kappa + x_b)),  kappa = c_ray / (c_path rho_mean),
 * rho_mean the mean returns per ray of a uniform launch; then mixed with the
 * uniform density as rr_proposal_build does.  A large kappa (rays dominate)
 * gives the square-root table (power 1/2); a small one (paths dominate) a
 * table flat over every direction that returns.  Errors as rr_proposal_build,
 * RR_EINVAL for kappa <= 0. */
int rr_proposal_build_cost(rr_ctx *ctx, const float *code16_dev, float beta, float kappa);

/* ------------------------------------------------------------------------
 * Batched launch: many scenes of uneven size (triangles, rays, channels,
 * chirps, samples) traced and synthesised (exact model) in one captured
 * launch.  One persistent trace kernel pulls (scene, chunk) items from a
 * device counter; synthesis runs per scene on one of two engines: the direct
 * FP32 engine (one persistent kernel over (scene, tile) items of every scene
 * that uses it) or the exact product engine of rr_synthesize's
 * RR_GEMM_EXACT (split-bf16 Tx x Rx products per sample on MFMA, kernels of
 * their own per scene, one scene after another on shared leg tables, each
 * reading its path range on the device).  Both meet the exact model's FP32
 * bar (relative error <= 1e-4).  The whole stage sequence is captured once as
 * a hipGraph and replayed; the engine, the product tile and the direct
 * engine's tile (samples per lane) per scene come from rr_batch_tune, or
 * from rr_batch_set_engine.
 * ------------------------------------------------------------------------ */
typedef struct rr_batch rr_batch;

/* A batch of n_scenes slots bound to ctx's device and stream. */
int rr_batch_create(rr_ctx *ctx, int32_t n_scenes, rr_batch **out);
void rr_batch_destroy(rr_batch *batch);

/* Fill slot `slot` with a scene (same arrays as rr_scene_upload), an array
 * (as rr_set_array), a chirp and trace parameters (uniform sampler only;
 * record_hits and path_cap are ignored).  Invalidates the captured graph. */
int rr_batch_set_scene(rr_batch *batch, int32_t slot, const float *verts, int64_t n_verts,
                       const int32_t *tris, const int32_t *tri_obj, int64_t n_tris,
                       const float *obj_alpha, const double *obj_vel, int32_t n_obj,
                       const double *pt_pos, const double *pt_vel, const double *pt_aperture,
                       int32_t n_pts, const double *tx, int32_t n_tx, const double *rx, int32_t n_rx,
                       double rx_radius, int32_t tx_mode, const rr_chirp *chirp,
                       const rr_trace_params *params);

/* As rr_scene_set_alpha for the scene in slot `slot` (per-object or per-face
 * alpha, Eq. 3); drains the batch's stream first.  The captured graph reads
 * the updated values on its next replay (no re-capture).
 * Errors: RR_EINVAL (slot, count, mode, range), RR_ESTATE (empty slot). */
int rr_batch_set_alpha(rr_batch *batch, int32_t slot, const float *alpha, int64_t n, int32_t per);

/* Run the batch: cubes[s] is scene s's complex64 [n_ch][n_chirps][n_samples]
 * device buffer.  The first launch (or the first after a change) captures the
 * pipeline as a hipGraph; later launches replay it (new cube pointers update
 * a device table, or re-capture when a scene uses the product engine).  The
 * call waits for completion and checks the path pool and the product
 * engine's leg-table capacity of every scene using it (sized from the
 * previous launch's count, else from the ray budget), growing them and
 * re-running if one overflowed.  n_paths_out (host int64 [n_scenes], may be
 * NULL) receives each scene's path count. */
int rr_batch_launch(rr_batch *batch, void *const *cubes, int64_t *n_paths_out);

/* Autotune the synthesis: run the batch once into `cubes` for its paths,
 * then, over at most the first 2048 paths of each path group (synthesis time
 * is linear in the path count): for every distinct sample count time each
 * candidate samples-per-lane value of the direct engine on the scenes with
 * that count and keep the fastest; then per scene left to RR_ENGINE_AUTO
 * time the direct engine against the product engine at every layout (the
 * sample split, tiles 16, 32, 48, 64, 96) whose modelled time (padded outputs
 * over the layout's measured throughput) is within 1.5x of the least (shared
 * launches only), and keep the product engine if it is faster by a tenth and
 * 20 us.  Afterwards
 * the cubes hold partial sums: run rr_batch_launch to fill them.
 * rr_batch_get_tiles reports the direct engine's samples per lane per scene;
 * rr_batch_get_plan the engine each scene runs on (RR_DIRECT_FP32 or
 * RR_GEMM_EXACT, both host int32 [n_scenes]) and its tile (samples per lane,
 * or the product layout as rr_batch_set_engine numbers it).  Untuned scenes
 * left to AUTO take rr_synthesize's rule (tables within 16 GiB). */
int rr_batch_tune(rr_batch *batch, void *const *cubes);
int rr_batch_get_tiles(rr_batch *batch, int32_t *samples_per_lane_out);
int rr_batch_get_plan(rr_batch *batch, int32_t *engine_out, int32_t *tile_out);

/* Pin slot `slot`'s synthesis engine: RR_ENGINE_AUTO (default: the tuner's
 * or the rule's choice), RR_DIRECT_FP32, or RR_GEMM_EXACT with product
 * layout `tile`: a square Tx x Rx tile of 16, 32, 48, 64 or 96, 1 for the
 * per-channel sample split (at most 1024 samples), 0 for the layout of least
 * modelled time.  Invalidates the captured graph.
 * Errors: RR_EINVAL (slot, engine, tile). */
int rr_batch_set_engine(rr_batch *batch, int32_t slot, int32_t engine, int32_t tile);

/* Timing (ms, HIP events around the graph launch) of the last launch, the
 * synthesis stage of the last autotuner run, and the last total path count. */
int rr_batch_stats(rr_batch *batch, double *ms_total, double *ms_synth, int64_t *total_paths);

/* ------------------------------------------------------------------------
 * Imaging (the paper forms images of its simulated data by brute-force
 * back-projection and shows their maximum projection in dB).
 * Voxel (i, j, k) is centred at (x0 + i step, y0 + j step, z0 + k step);
 * images are complex64 [nx][ny][nz] (x, the boresight range axis, slowest). */
typedef struct {
    double x0, y0, z0, step;
    int32_t nx, ny, nz;
} rr_volume;

/* Delay-and-sum back-projection of one sweep per channel: for every voxel x,
 *   image(x) = sum_{t, r} sum_k s[t n_rx + r][k] exp(+j 2 pi f_k d / c),
 *   d = |x - tx_t| + |x - rx_r|, f_k = f0 + B k / K (the context's chirp; a
 *   stepped-frequency sweep is one chirp of K steps),
 * the matched filter of the synthesis phase.  cube_dev: complex64
 * [n_ch][n_chirps][n_samples] as rr_synthesize writes it (chirp 0 of each
 * channel is used); image_dev: complex64, image_elems >= nx ny nz.
 * engine:
 *   RR_DIRECT_FP32  one lane per voxel: both legs and the phase reduction in
 *                   FP64 per (voxel, channel), the sum over frequencies by
 *                   Horner's rule in FP32 (at most 4096 steps);
 *   RR_GEMM_EXACT   per frequency, the Rx sum as a split-bf16 complex product
 *                   of the cube slice (Tx x Rx) with the Rx phasors of 128
 *                   voxels on the matrix cores, then the Tx sum on the vector
 *                   units; legs formed in FP64 and kept in FP32 (phases below
 *                   256 turns: volumes within ~0.9 m of the array at 80 GHz);
 *                   at most 96 Tx and 96 Rx;
 *   RR_ENGINE_AUTO  RR_GEMM_EXACT when it applies, else RR_DIRECT_FP32.
 * Both agree with the FP64 sum to ~1e-5 of the image's peak.  Errors:
 * RR_ESTATE (array or chirp missing), RR_EINVAL (sizes, grid, engine),
 * RR_EUNSUPPORTED (an engine's limits exceeded). */
int rr_backproject(rr_ctx *ctx, const void *cube_dev, int64_t cube_elems, const rr_volume *vol,
                   void *image_dev, int64_t image_elems, int32_t engine);

/* Maximum over x of |image| per (y, z), in dB relative to the largest of
 * them, clamped below at floor_db (e.g. -15): out_dev float [ny][nz].
 * Errors: RR_EINVAL. */
int rr_max_projection(rr_ctx *ctx, const void *image_dev, const rr_volume *vol, float *out_dev,
                      float floor_db);

/* Kernel timing of the last rr_trace / rr_synthesize / rr_backproject call,
 * in milliseconds, measured with HIP events on the context stream
 * (synchronises).  which: 0 = trace (all trace kernels, scan and scatter
 * included), 1 = synthesis main kernel, 2 = back-projection, 3 = the tracing
 * kernels of the last trace alone (the coherent ray order, rays and point
 * reflectors, before the scan). */
int rr_last_kernel_ms(rr_ctx *ctx, int32_t which, double *ms_out);

#ifdef __cplusplus
}
#endif

#endif /* RADRAY_H */
