/*
 * gr.h -- C ABI of libgr, the MI355X (gfx950) ray / 3D-Gaussian line-integral
 * projector.
 *
 * The library evaluates, for every ray r(t) = o + t d (t over the whole real
 * line, Eq. 3 of "Radioactive 3D Gaussian Ray Tracing for Tomographic
 * Reconstruction"), the order-free sum of exact line integrals through
 * anisotropic 3D Gaussians (Eq. 4 and the boxed Eq. 12):
 *
 *   I(o, d) = sum_i rho_i sqrt(2 pi / A_i) exp(-(C_i - B_i^2 / A_i) / 2),
 *   A = d^T P d,  B = d^T P (o - mu),  C = (o - mu)^T P (o - mu)   (Eq. 7),
 *
 * with P = Sigma^-1, Sigma = R S S^T R^T (Sec. 3.1), R the rotation of the
 * unit quaternion q / |q| = (w, x, y, z), S = diag(s), and rho the peak density
 * (the Gaussian normalisation is absorbed into rho, Eq. 2). The paper skips
 * "negligible" contributions without a rule (Sec. 4.1); here a pair counts iff
 * D = C - B^2/A <= kappa^2, i.e. the line meets the kappa-sigma ellipsoid.
 * It also provides the gradient of a per-ray loss with respect to every
 * Gaussian parameter (the paper optimises the parameters so that projections
 * match measurements, Fig. 1, but derives no gradient) and the ray set-up of
 * cone-/parallel-beam CT and arc-corrected PET (Fig. 1, Fig. 2, Sec. 3).
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers unless marked "host". Arrays are FP32
 *     and SoA: a [3n] array holds x[0..n), then y[0..n), then z[0..n); a [4n]
 *     quaternion array holds w, x, y, z blocks.
 *   - The library allocates no memory. Every buffer, including the
 *     acceleration-structure workspace and the backward scratch, is owned by
 *     the caller, who sizes it with the *_bytes queries. Buffers must be
 *     256-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the null stream). Every call only
 *     enqueues work on it and returns; the caller synchronises. Exceptions:
 *     gr_scene_invalid_count and gr_scene_status synchronise the stream.
 *   - Argument and size errors are detected on the host and returned before
 *     anything is enqueued. A HIP launch failure is returned as GR_E_HIP; a
 *     device fault from earlier asynchronous work makes later launches fail,
 *     so it surfaces as GR_E_HIP on a later call. No C++ exception crosses
 *     this interface.
 *   - The library must bind to the same HIP runtime instance as the caller
 *     (with PyTorch: import torch before loading libgr).
 *   - Calls are reentrant. Concurrent calls must not share output, scratch or
 *     workspace buffers that they write.
 */
#ifndef GR_H
#define GR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GR_ABI_VERSION 1

typedef int32_t gr_status;
enum {
    GR_OK = 0,
    GR_E_ARG = -1,         /* invalid argument (NULL pointer, bad size, bad enum, misalignment) */
    GR_E_WORKSPACE = -2,   /* workspace / scratch smaller than the *_bytes query */
    GR_E_HIP = -3,         /* a HIP runtime call or kernel launch failed */
    GR_E_UNSUPPORTED = -4, /* size beyond the library's limits (see GR_MAX_GAUSSIANS etc.) */
    GR_E_STATE = -5        /* workspace not built by gr_build_accel for this scene */
};

#define GR_MAX_GAUSSIANS (1LL << 28)
#define GR_MAX_LEAF_SIZE 64

/* Text for a status code (static storage, never NULL). */
const char *gr_status_str(gr_status status);
/* GR_ABI_VERSION of the loaded library. */
int32_t gr_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Scene and acceleration structure                                         */
/* ------------------------------------------------------------------------ */

/* A set of n Gaussians (Sec. 3.1, Eq. 2). mean[3n], scale[3n] (s > 0, the
 * standard deviations along the local axes), quat[4n] (w, x, y, z; need not be
 * unit), density[n] (peak density rho). kappa > 0 is the cutoff in standard
 * deviations (3 = the 3-sigma ellipsoid). leaf_size in [1, 64] is the number of
 * Morton-consecutive Gaussians per BVH leaf (0 = library default, 64).
 * accel / accel_bytes: caller-owned device workspace of at least
 * gr_accel_bytes(n, leaf_size) bytes. The parameter arrays must stay alive and
 * unchanged from gr_build_accel until the last gr_project_backward that uses
 * the scene (the backward epilogue reads scale and quat). */
typedef struct gr_scene {
    int64_t n;
    const float *mean;
    const float *scale;
    const float *quat;
    const float *density;
    float kappa;
    int32_t leaf_size;
    void *accel;
    size_t accel_bytes;
} gr_scene;

/* Bytes of acceleration workspace for n Gaussians and a leaf size (0 = default). */
gr_status gr_accel_bytes(int64_t n, int32_t leaf_size, size_t *bytes /* host */);

/* Builds the acceleration structure on the device, all on `stream`:
 * per-Gaussian preprocessing (rotation, whitening, kappa-sigma boxes,
 * validity), 30-bit Morton codes of the means inside the scene bounds, a
 * stable LSD radix sort, a Karras radix-tree LBVH over leaves of leaf_size
 * Gaussians with a bottom-up refit of the node boxes, and a 64-wide
 * hierarchy of boxes over the same Morton-ordered leaves. Gaussians with s <= 0,
 * q = 0 or non-finite values are counted and excluded from every result. */
gr_status gr_build_accel(const gr_scene *scene, void *stream);

/* Refit after the parameters changed in place (e.g. an optimiser step): the
 * Morton order and the tree topology of the last gr_build_accel on this
 * workspace are kept; every record, kappa box, node box and wide-hierarchy box
 * is recomputed from the current parameters, so results equal those of a full
 * build up to the order of summation. Cheaper than a build (no codes, no sort,
 * no tree), but the tree's quality decays as Gaussians move away from their
 * Morton positions: rebuild every few steps. kappa may change. The workspace
 * must hold a build for the same n and leaf_size; otherwise status bit 8 is
 * set (gr_scene_status) and results are undefined (the refit itself stays
 * inside the workspace). */
gr_status gr_refit_accel(const gr_scene *scene, void *stream);

/* Number of excluded (invalid) Gaussians. Synchronises `stream`. */
gr_status gr_scene_invalid_count(const gr_scene *scene, int64_t *n_invalid /* host */, void *stream);

/* Error bits recorded by the device-side consistency checks of the build and
 * of every traversal of this scene since the last build or refit (0 = none):
 * 1 = the tree is inconsistent, 2 = traversal stack overflow, 4 = traversal
 * step cap reached, 8 = refit of a workspace not built for this scene.
 * Non-zero means results computed with this scene are invalid.
 * Synchronises `stream`. */
gr_status gr_scene_status(const gr_scene *scene, int32_t *flags /* host */, void *stream);

/* ------------------------------------------------------------------------ */
/* Launch options                                                           */
/* ------------------------------------------------------------------------ */

/* Optional tuning knobs (NULL = defaults). A field set to 0 takes its default.
 * waves_per_group: waves (of 64 rays each) per workgroup, 1..16 (default 1).
 * xcd_remap: 1 (default) maps consecutive ray packets to the same XCD, 2
 *   disables the remap (grid launches only).
 * traversal: 2 (default) walks the 64-wide hierarchy over the Morton-ordered
 *   leaves, testing 64 child boxes against the packet's beam per wave step;
 *   1 walks the binary Karras LBVH with per-ray slab tests. Same results.
 * work_counter: NULL (default) launches one wave per 64-ray packet. A device
 *   pointer to one caller-owned uint32 selects the persistent launch:
 *   persistent_groups workgroups (0 = 20 waves per compute unit) loop, each
 *   wave taking the next packet from the counter with an atomic; the library
 *   zeroes the counter on the stream first. Concurrent calls need distinct
 *   counters. Results are identical to the grid launch.
 * hit_list_cap: hit-list entries per wave for the fused-loss backward (see
 *   gr_fused_scratch_bytes): 0 = default (8192), -1 = never record hit lists,
 *   else 64..1048576.
 * precision: the forward's arithmetic (gr_project, gr_project_stats,
 *   gr_project_batched; the other calls ignore it). 0 (default) evaluates
 *   Eq. 7 in FP64 from 80-byte records; 1 evaluates it in FP32 from 64-byte
 *   records (mean, whitening matrix diag(1/s) R^T, density): the offset o - mu
 *   is kept exactly as a sum of two floats, the line's origin is moved to the
 *   point nearest the mean, and D is the squared length of the whitened
 *   closest-point vector. A mixed-precision mode (Sec. 5 names mixed-precision
 *   computation among the ways to cut run time): same cutoff rule and FP64
 *   per-ray sum, larger rounding error (measured in the tests), and not
 *   faster on gfx950, where FP64 vector arithmetic runs at the unpacked FP32
 *   rate and the FP32 form needs about twice the instructions. */
typedef struct gr_launch {
    int32_t waves_per_group;
    int32_t xcd_remap;
    int32_t persistent_groups;
    int32_t traversal;
    uint32_t *work_counter;
    int32_t hit_list_cap;
    int32_t precision;
    int32_t reserved[2];
} gr_launch;

/* ------------------------------------------------------------------------ */
/* Forward projection                                                       */
/* ------------------------------------------------------------------------ */

/* out[r] = I(o_r, d_r) of Eq. 12 with the kappa cutoff, for n_rays rays
 * ray_o[3 n_rays], ray_d[3 n_rays]. d need not be unit length (the result is
 * the integral over the parameter t, so it scales as 1/|d|); d = 0 is invalid
 * and yields NaN or 0. Rays are processed in packets of 64 consecutive rays;
 * coherent packets (as written by the ray generators below) run fastest.
 * Summation order inside a ray is fixed, so the result is deterministic. */
gr_status gr_project(const gr_scene *scene, const float *ray_o, const float *ray_d, int64_t n_rays,
                     float *out, const gr_launch *opt, void *stream);

/* gr_project plus work counters, for measurement. The counters are ADDED to
 * stats[0..GR_STATS_COUNT) (device, uint64, 8-byte aligned; the caller zeroes;
 * entries beyond [5] are reserved):
 *   [0] included pairs (D <= kappa^2): the unit of the throughput metric,
 *   [1] evaluated (ray, Gaussian) pairs: candidate Gaussians x active rays
 *       of each packet (so [0]/[1] is the SIMD lane utilisation),
 *   [2] leaves visited, summed over packets,
 *   [3] packets,
 *   [4] candidate Gaussians (passed the packet's beam test), over packets,
 *   [5] candidates with at least one included pair in their packet.
 * out receives the same values as gr_project. */
#define GR_STATS_COUNT 8
gr_status gr_project_stats(const gr_scene *scene, const float *ray_o, const float *ray_d,
                           int64_t n_rays, float *out, uint64_t *stats, const gr_launch *opt,
                           void *stream);

/* Several ray segments, possibly against different scenes and different ray
 * arrays, in ONE launch. Each segment names a scene (index into scenes[]) and
 * its own SoA ray arrays ray_o[3 stride], ray_d[3 stride] (stride = the
 * length of each component block); it projects rays
 * [ray_offset, ray_offset + n_rays) into out[out_offset ...]. Each segment's
 * 64-ray packets start at its ray_offset, so its results equal gr_project on
 * those rays alone, bit for bit. The segment table is passed to the kernel by
 * value: at most GR_MAX_SEGMENTS segments and GR_MAX_SCENES scenes. */
#define GR_MAX_SEGMENTS 32
#define GR_MAX_SCENES 8
typedef struct gr_segment {
    int32_t scene;
    int32_t reserved;
    const float *ray_o;
    const float *ray_d;
    int64_t stride;
    int64_t ray_offset;
    int64_t n_rays;
    float *out;
    int64_t out_offset;
} gr_segment;
gr_status gr_project_batched(const gr_scene *scenes /* host, n_scenes */, int32_t n_scenes,
                             const gr_segment *segs /* host, n_segs */, int32_t n_segs,
                             const gr_launch *opt, void *stream);

/* ------------------------------------------------------------------------ */
/* Gradient                                                                 */
/* ------------------------------------------------------------------------ */

/* Loss fused into the backward pass (used when grad_out is NULL):
 *   GR_LOSS_L2:      L = 1/2 sum_r (I_r - target_r)^2,   dL/dI_r = I_r - target_r
 *   GR_LOSS_POISSON: L = sum_r (Ib_r - target_r log Ib_r), Ib_r = I_r + background,
 *                    dL/dI_r = 1 - target_r / Ib_r   (negative Poisson log-likelihood
 *                    up to a constant; PET counts are Poisson distributed, Sec. 2.1)
 * target[n_rays] (device). out_proj[n_rays] (optional, device) receives I.
 * out_loss (optional, device, one double) has L ADDED to it. */
enum { GR_LOSS_NONE = 0, GR_LOSS_L2 = 1, GR_LOSS_POISSON = 2 };
typedef struct gr_loss {
    int32_t kind;
    float background;
    const float *target;
    float *out_proj;
    double *out_loss;
} gr_loss;

/* Bytes of backward scratch for n Gaussians (10 FP32 accumulators each). */
gr_status gr_backward_scratch_bytes(int64_t n, size_t *bytes /* host */);

/* Bytes of scratch with which the fused-loss backward (grad_out NULL) runs
 * its hit-list form on the current device for launch options opt (may be
 * NULL): the accumulators, a work counter and one region of hit_list_cap
 * entries (12 bytes each) per persistent wave, persistent_groups x
 * waves_per_group waves (persistent_groups 0 = 20 waves per compute unit).
 * In that form the launch is persistent (using opt->work_counter if given,
 * else a counter in the scratch), the forward half records for every
 * candidate Gaussian with an included pair the 64-bit mask of its included
 * rays, and the backward half evaluates exactly those pairs, every lane busy,
 * instead of re-traversing. A packet whose list outgrows its region is
 * re-traversed. Results equal the re-traversal form's up to the order of the
 * FP32 atomics. With less scratch (but at least gr_backward_scratch_bytes)
 * the fused backward re-traverses. */
gr_status gr_fused_scratch_bytes(int64_t n, const gr_launch *opt, size_t *bytes /* host */);

/* Gradient of L with respect to the raw parameters of every Gaussian, where
 * dL/dI_r is grad_out[r] (or, if grad_out is NULL, comes from the fused loss).
 * Outputs (device, overwritten): grad_mean[3n], grad_scale[3n], grad_quat[4n]
 * (with respect to the raw, non-normalised q), grad_density[n]. Excluded
 * pairs (D > kappa^2) and invalid Gaussians contribute zero; the cutoff
 * indicator is held fixed. Nothing is stored between separate forward and
 * backward calls: with grad_out, candidates are found again by re-traversal;
 * the fused-loss form re-traverses or replays the hit lists of its own
 * forward half (gr_fused_scratch_bytes). FP32 atomics make the result
 * order-dependent at rounding level. scratch: caller-owned device buffer of
 * at least gr_backward_scratch_bytes(n) bytes, 256-byte aligned. */
gr_status gr_project_backward(const gr_scene *scene, const float *ray_o, const float *ray_d,
                              int64_t n_rays, const float *grad_out, const gr_loss *loss,
                              float *grad_mean, float *grad_scale, float *grad_quat,
                              float *grad_density, void *scratch, size_t scratch_bytes,
                              const gr_launch *opt, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Same as
 * gr_project_backward (same arguments, results equal to its up to the order
 * of the FP32 atomics) without the scratch arguments: the per-Gaussian sums,
 * the work counter and the hit lists live in a static device array of
 * GR_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs on until
 * the process ends. Nothing is allocated and nothing is freed. Hit lists get
 * the entries per wave that the array holds beside the sums (at most
 * hit_list_cap); with fewer than 64 the fused pass re-traverses. Limit: n with
 * 40 n + 512 <= GR_STATIC_SCRATCH_BYTES (about 3.3 million Gaussians), else
 * GR_E_UNSUPPORTED before anything is enqueued. Every call on a GPU shares
 * that GPU's array (each call clears what it needs zeroed first): calls that
 * overlap on one GPU (different streams or host threads without ordering)
 * race and give wrong results; serialise them. */
#define GR_STATIC_SCRATCH_BYTES (128u << 20)
gr_status gr_project_backward_static(const gr_scene *scene, const float *ray_o, const float *ray_d,
                                     int64_t n_rays, const float *grad_out, const gr_loss *loss,
                                     float *grad_mean, float *grad_scale, float *grad_quat,
                                     float *grad_density, const gr_launch *opt, void *stream);

/* The fused-loss pass split into chunks and batched across requests: the
 * gradient of a loss that is a sum over rays (both losses above are, Eq. 4
 * sums each ray's integrals in any order) is the sum of the gradients of any
 * partition of the rays, so a long request can be cut into runs of whole
 * 64-ray packets and the runs of several requests, against different scenes,
 * can share one launch. Each segment is one such run: rays
 * [ray_offset, ray_offset + n_rays) of SoA arrays ray_o[3 stride],
 * ray_d[3 stride] against scenes[scene], with its own fused loss (loss_kind
 * GR_LOSS_L2 or GR_LOSS_POISSON, background as gr_loss), targets
 * target[out_offset + i] for the segment's ray i, optional projection
 * out_proj[out_offset + i], optional out_loss (one double, the segment's loss
 * ADDED), and accum: the 10 x n FP32 per-Gaussian sums of its scene
 * (gr_backward_scratch_bytes(n) bytes, 256-byte aligned), ADDED to. Segments of
 * one request share its accum and loss. Each segment's packets start at its
 * ray_offset, so the projections equal those of gr_project_backward on the same
 * packets. */
typedef struct gr_bwd_segment {
    int32_t scene;
    int32_t loss_kind;
    const float *ray_o;
    const float *ray_d;
    int64_t stride;
    int64_t ray_offset;
    int64_t n_rays;
    const float *target;
    float *out_proj;
    int64_t out_offset;
    float *accum;
    double *out_loss;
    float background;
    int32_t reserved;
} gr_bwd_segment;

/* Zeroes the 10 x n accumulators of a request before its first segment. */
gr_status gr_backward_accum_zero(int64_t n, float *accum, void *stream);

/* One fused forward -> loss -> backward launch over up to GR_MAX_SEGMENTS
 * segments against up to GR_MAX_SCENES scenes (host arrays), accumulating into
 * each segment's accum; no epilogue. scratch: NULL (every packet re-traverses
 * for its backward half) or a device buffer, 256-byte aligned, of at least
 * gr_fused_scratch_bytes(0, opt) bytes holding the work counter and the
 * per-wave hit lists (hit_list_cap must not be -1). Concurrent calls need
 * distinct scratch; segments of concurrent calls must not share accum. */
gr_status gr_project_backward_batched(const gr_scene *scenes /* host, n_scenes */, int32_t n_scenes,
                                      const gr_bwd_segment *segs /* host, n_segs */, int32_t n_segs,
                                      void *scratch, size_t scratch_bytes, const gr_launch *opt, void *stream);

/* Chain rule from a request's accumulated sums to the raw parameter
 * gradients (the epilogue of gr_project_backward): outputs as
 * gr_project_backward, overwritten. accum as filled by the segments of
 * gr_project_backward_batched for this scene. */
gr_status gr_backward_finish(const gr_scene *scene, const float *accum, float *grad_mean, float *grad_scale,
                             float *grad_quat, float *grad_density, void *stream);

/* ------------------------------------------------------------------------ */
/* Ray generation (computed in FP64 on the device, rounded to FP32)         */
/* ------------------------------------------------------------------------ */

/* CT with rotation axis z (Fig. 1: ray origins and directions from the scanner
 * geometry). View v has angle th = angle0 + v * angle_range / n_views, source
 * direction e_s = (cos th, sin th, 0), detector axes e_u = (-sin th, cos th, 0)
 * and e_v = z; pixel (i, j) is at u = (i - (nu-1)/2) pitch_u + offset_u,
 * w = (j - (nv-1)/2) pitch_v + offset_v.
 *   cone = 0 (parallel beam): d = -e_s, o = u e_u + w e_v.
 *   cone = 1: source S = dso e_s, pixel P = -(dsd - dso) e_s + u e_u + w e_v,
 *             d = (P - S)/|P - S|, o = S - (S.d) d.
 * o is always the foot of the perpendicular from the isocentre and |d| = 1.
 * Ray order: view by view; inside a view the nu x nv pixel grid is cut into
 * tiles of tile_u x tile_v (edge tiles partial), enumerated tile row by tile
 * row, tile by tile, row-major inside a tile. With 8 x 8 tiles every 64-ray
 * packet is one detector tile. */
typedef struct gr_ct_geom {
    int32_t cone;
    int32_t n_views;
    int32_t nu;
    int32_t nv;
    double angle0;
    double angle_range;
    double dso;
    double dsd;
    double pitch_u;
    double pitch_v;
    double offset_u;
    double offset_v;
    int32_t tile_u;
    int32_t tile_v;
} gr_ct_geom;

/* Cylindrical PET: n_rings rings of n_crystals crystals on radius
 * ring_radius, ring z = (r - (n_rings-1)/2) ring_pitch. Radial index
 * k = kk - n_radial/2 for kk in [0, n_radial); view v in [0, n_views).
 * The line normal angle is psi = pi v / n_views + (k odd) pi / n_crystals and
 * the end points sit at angles psi +- (pi/2 - pi k / n_crystals) on rings r1
 * and r2: with arc_correct = 1 the line lies at its true chord distance
 * ring_radius sin(pi k / n_crystals), with non-uniform spacing, and both end
 * points are crystal centres when n_views = n_crystals/2 (Fig. 2; arc
 * correction applied at ray set-up, no sinogram resampling, Sec. 3 and 6).
 * arc_correct = 0 moves the same line in-plane along its normal to the
 * uniform distance k pi ring_radius / n_crystals (the straightened model).
 * Planes: planes (device, int32 pairs r1, r2, n_planes of them) or NULL for
 * all ordered ring pairs with |r1 - r2| <= max_ring_diff, grouped by ring
 * difference 0, +1, -1, +2, -2, ... and by r1 inside a group.
 * Ray order: views in blocks of tile_views consecutive views (0 or 1 = one
 * view per block; the last block may be shorter, V views); inside a block the
 * n_radial x n_planes grid (radial fastest) is tiled by tile_radial x
 * tile_axial like the CT grid, and each tile lists its cells for every view of
 * the block, view by view, row-major inside the tile. A shorter last block
 * whose V divides tile_views uses tiles tile_views / V times taller (in
 * planes), so that its tiles hold as many rays as the others. Packets are 64
 * consecutive rays: tiles of exactly 64 rays (tile_radial x tile_axial x
 * tile_views = 64, with n_radial and the plane count multiples of the tile)
 * keep every packet inside one tile; a packet that straddles two tiles can
 * span distant planes and runs far slower. 8 radial x 1 plane x 8 views holds
 * nearly coincident lines where they pass closest to the centre and runs the
 * 200k-Gaussian PET workload about twice as fast as 8 x 8 x 1. */
typedef struct gr_pet_geom {
    double ring_radius;
    double ring_pitch;
    int32_t n_crystals;
    int32_t n_rings;
    int32_t n_radial;
    int32_t n_views;
    int32_t max_ring_diff;
    int32_t arc_correct;
    const int32_t *planes;
    int32_t n_planes;
    int32_t tile_radial;
    int32_t tile_axial;
    int32_t tile_views;
} gr_pet_geom;

gr_status gr_rays_count_ct(const gr_ct_geom *g, int64_t *n_rays /* host */);
gr_status gr_rays_count_pet(const gr_pet_geom *g, int64_t *n_rays /* host */);
/* Writes ray_o[3 n_rays], ray_d[3 n_rays] (n_rays from the count query). */
gr_status gr_make_rays_ct(const gr_ct_geom *g, float *ray_o, float *ray_d, void *stream);
gr_status gr_make_rays_pet_arccorr(const gr_pet_geom *g, float *ray_o, float *ray_d, void *stream);

/* ------------------------------------------------------------------------ */
/* Reconstruction loop                                                      */
/* ------------------------------------------------------------------------ */

/* Grid of voxel centres origin + (ix, iy, iz) .* spacing (mm), ix fastest:
 * the voxel (ix, iy, iz) is element (iz * dims[1] + iy) * dims[0] + ix. */
typedef struct gr_grid {
    double origin[3];
    double spacing[3];  /* > 0 */
    int64_t dims[3];    /* >= 0, product <= 2^36 */
} gr_grid;

/* Voxelises a built scene: out[v] = sum over Gaussians with D <= kappa^2 of
 * rho exp(-D/2), D = (x_v - mu)^T Sigma^-1 (x_v - mu): the mixture density of
 * Eq. 2 at the voxel centres, with the projection's cutoff; the reconstructed
 * volume is the optimised Gaussians voxelised (Fig. 1). out: device FP32,
 * dims[0] dims[1] dims[2] elements, overwritten. D and the sum are FP64, the
 * exponential FP32; relative error <= 1e-5 per voxel. Invalid Gaussians
 * contribute nothing. opt is unused (may be NULL). */
gr_status gr_voxelize(const gr_scene *scene, const gr_grid *grid, float *out, const gr_launch *opt,
                      void *stream);

/* gr_voxelize plus work counters, for measurement. ADDED to stats[0..2)
 * (device, uint64, 8-byte aligned; the caller zeroes):
 *   [0] (voxel, Gaussian) pairs with D <= kappa^2: the unit of the
 *       voxelisation's throughput,
 *   [1] pairs evaluated (Gaussians whose kappa-box meets a 4x4x4 brick x the
 *       brick's voxels inside the grid).
 * out receives the same values as gr_voxelize. */
gr_status gr_voxelize_stats(const gr_scene *scene, const gr_grid *grid, float *out, uint64_t *stats,
                            const gr_launch *opt, void *stream);

/* One Adam step (the optimiser of Sec. 4.1) on count FP32 parameters, in
 * place: m <- beta1 m + (1 - beta1) g, v <- beta2 v + (1 - beta2) g^2,
 * p <- p - lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps).
 * param, m, v: device, updated; grad: device, read. step >= 1 counts the
 * calls on these moments; the caller zeroes m and v before step 1. */
typedef struct gr_adam {
    float lr;
    float beta1;
    float beta2;
    float eps;
    int64_t step;
} gr_adam;

gr_status gr_adam_step(float *param, const float *grad, float *m, float *v, int64_t count,
                       const gr_adam *hp, void *stream);

/* One Adam step on all parameters of a scene of n Gaussians in one launch.
 * Every array is 11 x n FP32 on the device, row-major, rows in the order
 * mean x, y, z (0-2), scale (3-5), quaternion w, x, y, z (6-9), density (10).
 *   theta:   the optimised variables, updated; rows 3-5 and 10 hold the
 *            natural logarithms of scale and density (they stay positive),
 *            the other rows the parameters themselves;
 *   grad:    dL/d(parameter) at `natural`, read: what gr_project_backward
 *            writes when its four gradient pointers address rows 0, 3, 6, 10;
 *   m, v:    Adam moments of theta, updated (the caller zeroes before step 1);
 *   natural: the parameters the projector consumes (a gr_scene whose four
 *            pointers address rows 0, 3, 6, 10), read for the chain rule of
 *            the log rows (dL/dlog x = x dL/dx), then overwritten with the
 *            updated values (exp of the log rows, the other rows copied).
 * The update of each row is gr_adam_step's with lr[group], group 0 = mean,
 * 1 = scale, 2 = quaternion, 3 = density. The five arrays must not overlap. */
typedef struct gr_gauss_adam {
    float lr[4];
    float beta1;
    float beta2;
    float eps;
    int32_t reserved;
    int64_t step;
} gr_gauss_adam;

gr_status gr_adam_gaussians(int64_t n, float *theta, const float *grad, float *m, float *v, float *natural,
                            const gr_gauss_adam *hp, void *stream);

/* ------------------------------------------------------------------------ */
/* Time of flight, attenuation, randoms and scatter (PET)                    */
/* ------------------------------------------------------------------------ */

/* The paper names attenuation, scatter, randoms and time-of-flight PET as the
 * projector's next extensions (Sec. 5, future works). Model of one line r:
 * TOF bin b weighs the line by the kernel
 *   h_b(t) = (bin_width / (sqrt(2 pi) sigma)) exp(-(t - tau_b)^2 / (2 sigma^2)),
 *   tau_b  = center[r] + (b - (n_bins - 1) / 2) bin_width,
 * t the ray parameter (mm along a unit direction), and atten[r] multiplies
 * every bin:  I_b(r) = atten[r] sum_i rho_i Int G_i(o + t d) h_b(t) dt.
 * The Gaussian's and the kernel's exponents are both quadratic in t, so the
 * integral keeps Eq. 11's closed form with A' = A + 1/sigma^2,
 * B' = B - tau_b/sigma^2, C' = C + tau_b^2/sigma^2. A pair counts as in
 * gr_project (D <= kappa^2). Randoms and scatter enter the loss as additive
 * expected counts (gr_loss_weights).
 *   n_bins:    0 = no TOF kernel (one output per ray: atten times the
 *              projection), else 1..GR_TOF_MAX_BINS;
 *   sigma:     kernel standard deviation, 1e-12 <= sigma with sigma^2 <= 3e38
 *              (else GR_E_ARG; the FWHM of the timing resolution in mm is
 *              c dt / 2, sigma = FWHM / 2.3548);
 *   bin_width: spacing of the bin centres, > 0;
 *   center:    device FP32 per ray (the centre bin's t), or NULL for 0; for
 *              PET lines from gr_make_rays_pet_arccorr use gr_tof_centers;
 *   atten:     device FP32 per ray, or NULL for 1.
 * Outputs and weights are bin-major: element b * n_rays + r, with
 * max(1, n_bins) rows. Relative error <= 1e-5 per (ray, bin) against FP64. */
#define GR_TOF_MAX_BINS 32
typedef struct gr_tof {
    int32_t n_bins;
    float sigma;
    float bin_width;
    int32_t reserved;
    const float *center;
    const float *atten;
} gr_tof;

/* Forward: out[max(1, n_bins) * n_rays] (device FP32), overwritten. Rays as
 * gr_project; opt as gr_project with at most 4 waves per group
 * (hit_list_cap unused). */
gr_status gr_project_tof(const gr_scene *scene, const float *ray_o, const float *ray_d, int64_t n_rays,
                         const gr_tof *tof, float *out, const gr_launch *opt, void *stream);

/* Gradient of L = sum_{b, r} grad_out[b n_rays + r] I_b(r) with respect to
 * the raw parameters (outputs as gr_project_backward). scratch as
 * gr_project_backward with dL/dI given: at least gr_backward_scratch_bytes(n)
 * bytes, 256-byte aligned. Rays whose weights are all zero cost nothing. */
gr_status gr_project_tof_backward(const gr_scene *scene, const float *ray_o, const float *ray_d, int64_t n_rays,
                                  const gr_tof *tof, const float *grad_out, float *grad_mean, float *grad_scale,
                                  float *grad_quat, float *grad_density, void *scratch, size_t scratch_bytes,
                                  const gr_launch *opt, void *stream);

/* TOF centre of each ray: the parameter where it passes closest to the z
 * axis in the transaxial plane, -(o_xy . d_xy) / |d_xy|^2 (0 if d_xy = 0).
 * For a PET line with both end points on the detector cylinder this is the
 * midpoint of the end points, where the two photons' arrival times are equal.
 * ray_o, ray_d: device SoA as gr_project; center: device FP32 [n_rays]. */
gr_status gr_tof_centers(const float *ray_o, const float *ray_d, int64_t n_rays, float *center, void *stream);

/* Per-measurement loss weights w = dL/dI and the loss, for a projection proj
 * (any layout: count elements) and measurements target:
 *   GR_LOSS_L2:      L = sum (I - y)^2 / 2,            w = I - y;
 *   GR_LOSS_POISSON: L = sum (Ib - y log Ib), Ib = I + b, w = 1 - y / Ib,
 * b = background[i] (device FP32, the expected randoms + scatter counts of
 * element i; every Ib must be > 0) or background_scalar (> 0) when background
 * is NULL. weight: device FP32 [count], overwritten. loss: device FP64, 8-byte
 * aligned, the loss is ADDED to it (may be NULL). */
gr_status gr_loss_weights(int32_t kind, const float *proj, const float *target, const float *background,
                          float background_scalar, int64_t count, float *weight, double *loss, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GR_H */
