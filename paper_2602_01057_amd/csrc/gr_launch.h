// Launch tables shared by the projection kernels and the C ABI layer.
#pragma once

#include "gr_internal.h"

namespace gr {

// One contiguous run of rays against one scene. Packets of 64 rays never
// straddle two segments; first_packet is filled in by the host driver. The
// fused-loss backward reads its loss, targets and accumulators per segment, so
// that one launch can serve chunks of several requests.
struct Segment {
    int32_t scene;
    int32_t loss_kind;  // fused backward: GR_LOSS_L2 / GR_LOSS_POISSON
    const float *ro;    // SoA ray arrays of the segment, component stride `stride`
    const float *rd;
    int64_t stride;
    int64_t ray_offset;
    int64_t n_rays;
    float *out;         // forward output; fused backward: the projection (optional)
    int64_t out_offset; // ray i of the segment writes out[out_offset + i], reads target[...] there
    int64_t first_packet;
    const float *target;  // fused backward: targets / counts
    float *acc;           // fused backward: 10 x n accumulators of the segment's scene (Morton order)
    double *loss;         // fused backward: the loss is added here (optional)
    float background;     // fused backward: Poisson background
    int32_t pad;
};

// Passed by value as a kernel argument (well under the kernarg limit).
struct LaunchTable {
    SceneView scenes[GR_MAX_SCENES];
    Segment segs[GR_MAX_SEGMENTS];
    int32_t n_segs;
    int32_t waves_per_group;
    int32_t xcd_remap;
    int32_t persistent_groups;
    int64_t n_packets;
    uint32_t *work_counter;  // non-NULL: persistent launch
    int32_t traversal;       // 1 binary LBVH, 2 wide hierarchy
    int32_t precision;       // forward: 0 FP64 quadratic forms, 1 compact FP32 records
    int32_t hit_cap;         // > 0: fused backward records hit lists (persistent only)
    uint32_t *hit_g;         // per-wave-slot regions of hit_cap entries each
    uint64_t *hit_m;
};

// Backward launch arguments beside the table: dL/dI given (grad_out, the
// accumulators acc) or, with grad_out NULL, the fused loss whose fields sit in
// the segments.
struct BwdArgs {
    const float *grad_out;  // NULL in fused-loss mode
    float *acc;             // 10 x n accumulators (Morton order) of the dL/dI-given form
};

// Kernel arguments are limited to 4 KiB.
static_assert(sizeof(LaunchTable) + sizeof(BwdArgs) <= 4096, "kernel arguments exceed 4 KiB");

// Launch shape resolved from gr_launch.
struct LaunchShape {
    int waves;
    int remap;
    int persistent_groups;
    int traversal;
    uint32_t *work_counter;
    int hit_cap;  // hit-list entries per wave for the fused backward (0 = re-traverse)
    int precision;  // forward only: 0 FP64 (default), 1 compact FP32 records
};

hipError_t enqueue_forward(LaunchTable &T, const LaunchShape &shape, hipStream_t st,
                           uint64_t *stats = nullptr);
// hit_g / hit_m: hit-list regions (persistent_groups x waves of shape.hit_cap
// entries) when the fused pass records hit lists, else NULL.
hipError_t enqueue_backward(LaunchTable &T, const BwdArgs &A, const gr_scene &sc, const uint32_t *order,
                            float *gmean, float *gscale, float *gquat, float *gdens,
                            const LaunchShape &shape, uint32_t *hit_g, uint64_t *hit_m,
                            hipStream_t st);
// The fused-loss pass alone over the table's segments (each with its own loss
// fields and accumulators): no zeroing of the accumulators, no epilogue.
hipError_t enqueue_fused_segments(LaunchTable &T, const LaunchShape &shape, uint32_t *hit_g, uint64_t *hit_m,
                                  hipStream_t st);

// Packet numbering of the segments and the launch shape, filled in before a
// launch.
inline void finish_table(LaunchTable &T, const LaunchShape &shape) {
    int64_t pk = 0;
    for (int s = 0; s < T.n_segs; ++s) {
        T.segs[s].first_packet = pk;
        pk += (T.segs[s].n_rays + 63) / 64;
    }
    T.n_packets = pk;
    T.waves_per_group = shape.waves;
    T.xcd_remap = shape.remap;
    T.persistent_groups = shape.persistent_groups;
    T.work_counter = shape.work_counter;
    T.traversal = shape.traversal;
    T.precision = shape.precision;
}

// Workgroups of a launch: one wave per packet, or the persistent count.
inline unsigned launch_groups(const LaunchTable &T, const LaunchShape &shape) {
    if (shape.work_counter) return unsigned(shape.persistent_groups);
    return unsigned((T.n_packets + shape.waves - 1) / shape.waves);
}

// Zero-fill kernels (capturable in a graph, unlike a memset node).
void enqueue_zero_f32(float *p, int64_t count, hipStream_t st);
void enqueue_zero_u32(uint32_t *p, hipStream_t st);
// Chain rule from the 10 x n per-Gaussian sums (Morton order) to the raw
// parameter gradients (input order).
void enqueue_epilogue(const gr_scene &sc, const uint32_t *order, const float *acc, float *gmean, float *gscale,
                      float *gquat, float *gdens, hipStream_t st);

// Time-of-flight / attenuation model of one launch (bin-major outputs and
// weights [nb][n_rays], nb = max(1, n_bins); per-ray arrays indexed like the
// rays of the single segment).
struct TofArgs {
    int32_t n_bins;        // 0: no TOF kernel
    float sigma2;          // TOF kernel variance along the ray parameter
    float width;           // bin spacing
    float pad;
    const float *center;   // per ray, or NULL (0)
    const float *atten;    // per ray, or NULL (1)
    int64_t n_rays;        // stride of the bins
    float *out;            // forward output
    const float *grad_out; // backward weights dL/dI
    float *acc;            // backward: 10 x n accumulators (Morton order)
};

hipError_t enqueue_forward_tof(LaunchTable &T, const TofArgs &A, const LaunchShape &shape, hipStream_t st);
hipError_t enqueue_backward_tof(LaunchTable &T, const TofArgs &A, const gr_scene &sc, const uint32_t *order,
                                float *gmean, float *gscale, float *gquat, float *gdens, const LaunchShape &shape,
                                hipStream_t st);
hipError_t enqueue_tof_centers(const float *ro, const float *rd, int64_t n, float *center, hipStream_t st);
hipError_t enqueue_loss_weights(int32_t kind, const float *proj, const float *target, const float *bg_arr,
                                float bg, int64_t count, float *weight, double *loss, hipStream_t st);

}  // namespace gr
