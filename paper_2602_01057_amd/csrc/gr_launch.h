// Launch tables shared by the projection kernels and the C ABI layer.
#pragma once

#include "gr_internal.h"

namespace gr {

// One contiguous run of rays against one scene. Packets of 64 rays never
// straddle two segments; first_packet is filled in by the host driver.
struct Segment {
    int32_t scene;
    int32_t pad;
    const float *ro;  // SoA ray arrays of the segment, component stride `stride`
    const float *rd;
    int64_t stride;
    int64_t ray_offset;
    int64_t n_rays;
    float *out;       // forward output (NULL in backward launches)
    int64_t out_offset;
    int64_t first_packet;
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
    int32_t hit_cap;         // > 0: fused backward records hit lists (persistent only)
    uint32_t *hit_g;         // per-wave-slot regions of hit_cap entries each
    uint64_t *hit_m;
};

struct BwdArgs {
    const float *grad_out;  // NULL in fused-loss mode
    float *acc;             // 10 x n accumulators (Morton order)
    int32_t loss_kind;
    float background;
    const float *target;
    float *out_proj;
    double *out_loss;
};

// Launch shape resolved from gr_launch.
struct LaunchShape {
    int waves;
    int remap;
    int persistent_groups;
    int traversal;
    uint32_t *work_counter;
    int hit_cap;  // hit-list entries per wave for the fused backward (0 = re-traverse)
};

hipError_t enqueue_forward(LaunchTable &T, const LaunchShape &shape, hipStream_t st,
                           uint64_t *stats = nullptr);
// hit_g / hit_m: hit-list regions (persistent_groups x waves of shape.hit_cap
// entries) when the fused pass records hit lists, else NULL.
hipError_t enqueue_backward(LaunchTable &T, const BwdArgs &A, const gr_scene &sc, const uint32_t *order,
                            float *gmean, float *gscale, float *gquat, float *gdens,
                            const LaunchShape &shape, uint32_t *hit_g, uint64_t *hit_m,
                            hipStream_t st);

}  // namespace gr
