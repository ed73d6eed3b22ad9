// C ABI of libgr: argument validation, workspace sizing and launch set-up.
// Every check happens on the host before anything is enqueued.
#include <math.h>
#include <string.h>

#include <mutex>

#include "gr_internal.h"

namespace gr {
hipError_t enqueue_build(const gr_scene &sc, const Layout &L, hipStream_t st);
hipError_t enqueue_refit(const gr_scene &sc, const Layout &L, hipStream_t st);
int64_t pet_default_plane_count(int n_rings, int max_diff);
hipError_t enqueue_voxelize(const SceneView &S, const gr_grid &g, float *out, uint64_t *stats, hipStream_t st);
hipError_t enqueue_adam_gaussians(int64_t n, float *theta, const float *grad, float *m, float *v, float *natural,
                                  const gr_gauss_adam &hp, hipStream_t st);
hipError_t enqueue_adam(float *p, const float *g, float *m, float *v, int64_t count, const gr_adam &hp,
                        hipStream_t st);
hipError_t enqueue_rays_ct(const gr_ct_geom &g, int64_t n, float *ro, float *rd, hipStream_t st);
hipError_t enqueue_rays_pet(const gr_pet_geom &g, int64_t n_planes, int64_t n, float *ro, float *rd,
                            hipStream_t st);
}  // namespace gr

#include "gr_launch.h"

using namespace gr;

namespace {

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

gr_status map_hip(hipError_t e) { return e == hipSuccess ? GR_OK : GR_E_HIP; }

// Clears the thread's last-error slot, which other libraries' failed calls
// may have left set, so that the hipGetLastError after our launches reports
// only our own launch failures. A device fault from earlier asynchronous work
// is sticky: our launches then fail and the call returns GR_E_HIP.
gr_status pending_error() {
    (void)hipGetLastError();
    return GR_OK;
}

int32_t resolve_leaf(int32_t leaf) { return leaf == 0 ? kDefaultLeaf : leaf; }

gr_status check_scene(const gr_scene *s, bool need_accel) {
    if (!s) return GR_E_ARG;
    if (s->n < 0) return GR_E_ARG;
    if (s->n > GR_MAX_GAUSSIANS) return GR_E_UNSUPPORTED;
    const int32_t leaf = resolve_leaf(s->leaf_size);
    if (leaf < 1 || leaf > GR_MAX_LEAF_SIZE) return GR_E_ARG;
    if (!(s->kappa > 0.0f) || !isfinite(s->kappa)) return GR_E_ARG;
    if (s->n > 0 && (!s->mean || !s->scale || !s->quat || !s->density)) return GR_E_ARG;
    if (need_accel) {
        if (!s->accel || !aligned(s->accel, 256)) return GR_E_ARG;
        const Layout L = make_layout(s->n, leaf);
        if (s->accel_bytes < L.total) return GR_E_WORKSPACE;
    }
    return GR_OK;
}

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

gr_status check_launch(const gr_launch *opt, LaunchShape &sh) {
    sh.waves = 1;
    sh.remap = 1;
    sh.persistent_groups = 0;
    sh.traversal = 2;
    sh.work_counter = nullptr;
    sh.hit_cap = kDefaultHitCap;
    sh.precision = 0;
    if (!opt) return GR_OK;
    if (opt->precision != 0 && opt->precision != 1) return GR_E_ARG;
    sh.precision = opt->precision;
    if (opt->hit_list_cap == -1) sh.hit_cap = 0;
    else if (opt->hit_list_cap != 0) {
        if (opt->hit_list_cap < 64 || opt->hit_list_cap > (1 << 20)) return GR_E_ARG;
        sh.hit_cap = opt->hit_list_cap;
    }
    if (opt->traversal) sh.traversal = opt->traversal;
    if (sh.traversal != 1 && sh.traversal != 2) return GR_E_ARG;
    if (opt->waves_per_group) sh.waves = opt->waves_per_group;
    if (opt->xcd_remap) sh.remap = opt->xcd_remap;
    if (sh.waves < 1 || sh.waves > 16 || (sh.remap != 1 && sh.remap != 2)) return GR_E_ARG;
    if (opt->persistent_groups < 0) return GR_E_ARG;
    if (opt->work_counter) {
        if (!aligned(opt->work_counter, 4)) return GR_E_ARG;
        sh.work_counter = opt->work_counter;
        sh.persistent_groups = opt->persistent_groups;
        if (sh.persistent_groups == 0) sh.persistent_groups = (device_cu_count() * 20 + sh.waves - 1) / sh.waves;
    }
    return GR_OK;
}

gr_status check_ct(const gr_ct_geom *g) {
    if (!g) return GR_E_ARG;
    if (g->cone != 0 && g->cone != 1) return GR_E_ARG;
    if (g->n_views < 0 || g->nu < 0 || g->nv < 0) return GR_E_ARG;
    if (g->tile_u < 1 || g->tile_v < 1) return GR_E_ARG;
    if (!isfinite(g->angle0) || !isfinite(g->angle_range) || !isfinite(g->pitch_u) ||
        !isfinite(g->pitch_v) || !isfinite(g->offset_u) || !isfinite(g->offset_v))
        return GR_E_ARG;
    if (g->cone == 1 && !(g->dso > 0.0 && g->dsd > g->dso && isfinite(g->dsd))) return GR_E_ARG;
    return GR_OK;
}

gr_status check_pet(const gr_pet_geom *g, int64_t &n_planes) {
    if (!g) return GR_E_ARG;
    if (!(g->ring_radius > 0.0) || !isfinite(g->ring_radius) || !isfinite(g->ring_pitch)) return GR_E_ARG;
    if (g->n_crystals < 2 || g->n_rings < 1 || g->n_radial < 0 || g->n_views < 0) return GR_E_ARG;
    if (g->max_ring_diff < 0 || (g->arc_correct != 0 && g->arc_correct != 1)) return GR_E_ARG;
    if (g->tile_radial < 1 || g->tile_axial < 1 || g->tile_views < 0) return GR_E_ARG;
    if (g->planes) {
        if (g->n_planes < 0) return GR_E_ARG;
        n_planes = g->n_planes;
    } else {
        n_planes = pet_default_plane_count(g->n_rings, g->max_ring_diff);
    }
    // |k| pi / N must stay below pi/2 for the chord to exist
    if (2 * int64_t(g->n_radial / 2 + 1) > int64_t(g->n_crystals)) return GR_E_ARG;
    return GR_OK;
}

}  // namespace

extern "C" {

const char *gr_status_str(gr_status s) {
    switch (s) {
        case GR_OK: return "ok";
        case GR_E_ARG: return "invalid argument";
        case GR_E_WORKSPACE: return "workspace or scratch buffer too small";
        case GR_E_HIP: return "HIP runtime error";
        case GR_E_UNSUPPORTED: return "size beyond library limits";
        case GR_E_STATE: return "workspace not built for this scene";
        default: return "unknown status";
    }
}

int32_t gr_abi_version(void) { return GR_ABI_VERSION; }

gr_status gr_accel_bytes(int64_t n, int32_t leaf_size, size_t *bytes) {
    if (!bytes || n < 0) return GR_E_ARG;
    if (n > GR_MAX_GAUSSIANS) return GR_E_UNSUPPORTED;
    const int32_t leaf = resolve_leaf(leaf_size);
    if (leaf < 1 || leaf > GR_MAX_LEAF_SIZE) return GR_E_ARG;
    *bytes = make_layout(n, leaf).total;
    return GR_OK;
}

gr_status gr_build_accel(const gr_scene *scene, void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if ((st = pending_error()) != GR_OK) return st;
    const Layout L = make_layout(scene->n, resolve_leaf(scene->leaf_size));
    return map_hip(enqueue_build(*scene, L, static_cast<hipStream_t>(stream)));
}

gr_status gr_refit_accel(const gr_scene *scene, void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if ((st = pending_error()) != GR_OK) return st;
    const Layout L = make_layout(scene->n, resolve_leaf(scene->leaf_size));
    return map_hip(enqueue_refit(*scene, L, static_cast<hipStream_t>(stream)));
}

gr_status gr_scene_invalid_count(const gr_scene *scene, int64_t *n_invalid, void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if (!n_invalid) return GR_E_ARG;
    AccelHeader h;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(&h, scene->accel, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess)
        return GR_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return GR_E_HIP;
    if (h.magic != kMagic || !h.built || h.n != scene->n) return GR_E_STATE;
    *n_invalid = h.n_invalid;
    return GR_OK;
}

gr_status gr_scene_status(const gr_scene *scene, int32_t *flags, void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if (!flags) return GR_E_ARG;
    AccelHeader h;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(&h, scene->accel, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess)
        return GR_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return GR_E_HIP;
    if (h.magic != kMagic || !h.built || h.n != scene->n) return GR_E_STATE;
    *flags = h.flags;
    return GR_OK;
}

static gr_status project_impl(const gr_scene *scene, const float *ray_o, const float *ray_d,
                              int64_t n_rays, float *out, uint64_t *stats, const gr_launch *opt,
                              void *stream);

gr_status gr_project(const gr_scene *scene, const float *ray_o, const float *ray_d, int64_t n_rays,
                     float *out, const gr_launch *opt, void *stream) {
    return project_impl(scene, ray_o, ray_d, n_rays, out, nullptr, opt, stream);
}

gr_status gr_project_stats(const gr_scene *scene, const float *ray_o, const float *ray_d,
                           int64_t n_rays, float *out, uint64_t *stats, const gr_launch *opt,
                           void *stream) {
    if (!stats || !aligned(stats, 8)) return GR_E_ARG;
    return project_impl(scene, ray_o, ray_d, n_rays, out, stats, opt, stream);
}

static gr_status project_impl(const gr_scene *scene, const float *ray_o, const float *ray_d,
                              int64_t n_rays, float *out, uint64_t *stats, const gr_launch *opt,
                              void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if (n_rays < 0) return GR_E_ARG;
    if (n_rays > 0 && (!ray_o || !ray_d || !out)) return GR_E_ARG;
    if (n_rays > (int64_t(1) << 40)) return GR_E_UNSUPPORTED;
    LaunchShape shape;
    if ((st = check_launch(opt, shape)) != GR_OK) return st;
    if ((st = pending_error()) != GR_OK) return st;
    LaunchTable T;
    memset(&T, 0, sizeof(T));
    const Layout L = make_layout(scene->n, resolve_leaf(scene->leaf_size));
    T.scenes[0] = make_view(*scene, L);
    T.n_segs = 1;
    T.segs[0].scene = 0;
    T.segs[0].ro = ray_o;
    T.segs[0].rd = ray_d;
    T.segs[0].stride = n_rays;
    T.segs[0].ray_offset = 0;
    T.segs[0].n_rays = n_rays;
    T.segs[0].out = out;
    T.segs[0].out_offset = 0;
    return map_hip(enqueue_forward(T, shape, static_cast<hipStream_t>(stream), stats));
}

gr_status gr_project_batched(const gr_scene *scenes, int32_t n_scenes, const gr_segment *segs,
                             int32_t n_segs, const gr_launch *opt, void *stream) {
    if (!scenes || n_scenes < 1 || n_segs < 0 || (n_segs > 0 && !segs)) return GR_E_ARG;
    if (n_scenes > GR_MAX_SCENES || n_segs > GR_MAX_SEGMENTS) return GR_E_UNSUPPORTED;
    gr_status st;
    for (int s = 0; s < n_scenes; ++s)
        if ((st = check_scene(&scenes[s], true)) != GR_OK) return st;
    for (int k = 0; k < n_segs; ++k) {
        const gr_segment &g = segs[k];
        if (g.scene < 0 || g.scene >= n_scenes || g.ray_offset < 0 || g.n_rays < 0 ||
            g.out_offset < 0 || g.stride < 0 || g.ray_offset + g.n_rays > g.stride)
            return GR_E_ARG;
        if (g.n_rays > 0 && (!g.ray_o || !g.ray_d || !g.out)) return GR_E_ARG;
    }
    LaunchShape shape;
    if ((st = check_launch(opt, shape)) != GR_OK) return st;
    if ((st = pending_error()) != GR_OK) return st;
    LaunchTable T;
    memset(&T, 0, sizeof(T));
    for (int s = 0; s < n_scenes; ++s) {
        const Layout L = make_layout(scenes[s].n, resolve_leaf(scenes[s].leaf_size));
        T.scenes[s] = make_view(scenes[s], L);
    }
    T.n_segs = n_segs;
    for (int k = 0; k < n_segs; ++k) {
        T.segs[k].scene = segs[k].scene;
        T.segs[k].ro = segs[k].ray_o;
        T.segs[k].rd = segs[k].ray_d;
        T.segs[k].stride = segs[k].stride;
        T.segs[k].ray_offset = segs[k].ray_offset;
        T.segs[k].n_rays = segs[k].n_rays;
        T.segs[k].out = segs[k].out;
        T.segs[k].out_offset = segs[k].out_offset;
    }
    return map_hip(enqueue_forward(T, shape, static_cast<hipStream_t>(stream)));
}

gr_status gr_backward_scratch_bytes(int64_t n, size_t *bytes) {
    if (!bytes || n < 0) return GR_E_ARG;
    if (n > GR_MAX_GAUSSIANS) return GR_E_UNSUPPORTED;
    *bytes = align256(size_t(10) * size_t(n > 0 ? n : 1) * sizeof(float));
    return GR_OK;
}

namespace {

// Scratch layout of the fused backward's hit-list form: accumulators, work
// counter, then the per-wave regions (Gaussian indices, then masks).
struct FusedLayout {
    size_t counter, hit_g, hit_m, total;
    int groups;
};

gr_status fused_layout(int64_t n, const gr_launch *opt, const LaunchShape &sh, FusedLayout &F) {
    size_t acc = 0;
    gr_status st = gr_backward_scratch_bytes(n, &acc);
    if (st != GR_OK) return st;
    F.groups = (opt && opt->persistent_groups > 0) ? opt->persistent_groups
                                                   : (device_cu_count() * 20 + sh.waves - 1) / sh.waves;
    const size_t waves = size_t(F.groups) * size_t(sh.waves);
    const size_t entries = waves * size_t(sh.hit_cap > 0 ? sh.hit_cap : 0);
    F.counter = acc;
    F.hit_g = F.counter + 256;
    F.hit_m = F.hit_g + align256(entries * sizeof(uint32_t));
    F.total = F.hit_m + align256(entries * sizeof(uint64_t));
    return GR_OK;
}

}  // namespace

gr_status gr_fused_scratch_bytes(int64_t n, const gr_launch *opt, size_t *bytes) {
    if (!bytes) return GR_E_ARG;
    LaunchShape sh;
    gr_status st = check_launch(opt, sh);
    if (st != GR_OK) return st;
    FusedLayout F;
    if ((st = fused_layout(n, opt, sh, F)) != GR_OK) return st;
    if (sh.hit_cap == 0) return gr_backward_scratch_bytes(n, bytes);
    *bytes = F.total;
    return GR_OK;
}

}  // extern "C"

namespace {

// The backward of gr_project_backward with the launch shape already resolved
// (shape.hit_cap may be lowered by the caller to what the scratch holds).
gr_status backward_common(const gr_scene *scene, const float *ray_o, const float *ray_d, int64_t n_rays,
                          const float *grad_out, const gr_loss *loss, float *grad_mean, float *grad_scale,
                          float *grad_quat, float *grad_density, void *scratch, size_t scratch_bytes,
                          LaunchShape shape, const gr_launch *opt, void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if (n_rays < 0) return GR_E_ARG;
    if (n_rays > 0 && (!ray_o || !ray_d)) return GR_E_ARG;
    if (scene->n > 0 && (!grad_mean || !grad_scale || !grad_quat || !grad_density)) return GR_E_ARG;
    LaunchTable T;
    memset(&T, 0, sizeof(T));
    BwdArgs A{nullptr, nullptr};
    if (grad_out) {
        A.grad_out = grad_out;
        if (loss && loss->kind != GR_LOSS_NONE) return GR_E_ARG;
    } else {
        if (!loss || (loss->kind != GR_LOSS_L2 && loss->kind != GR_LOSS_POISSON)) return GR_E_ARG;
        if (n_rays > 0 && !loss->target) return GR_E_ARG;
        if (!isfinite(loss->background)) return GR_E_ARG;
        if (loss->kind == GR_LOSS_POISSON && !(loss->background > 0.0f)) return GR_E_ARG;
        T.segs[0].loss_kind = loss->kind;
        T.segs[0].background = loss->background;
        T.segs[0].target = loss->target;
        T.segs[0].out = loss->out_proj;
        T.segs[0].loss = loss->out_loss;
    }
    size_t need = 0;
    gr_backward_scratch_bytes(scene->n, &need);
    if (!scratch || !aligned(scratch, 256)) return GR_E_ARG;
    if (scratch_bytes < need) return GR_E_WORKSPACE;
    if ((st = pending_error()) != GR_OK) return st;
    A.acc = static_cast<float *>(scratch);
    T.segs[0].acc = A.acc;
    // hit-list form of the fused pass when the scratch holds the regions
    uint32_t *hit_g = nullptr;
    uint64_t *hit_m = nullptr;
    if (!grad_out && shape.hit_cap > 0) {
        FusedLayout F;
        if ((st = fused_layout(scene->n, opt, shape, F)) != GR_OK) return st;
        if (scratch_bytes >= F.total) {
            char *base = static_cast<char *>(scratch);
            if (!shape.work_counter) shape.work_counter = reinterpret_cast<uint32_t *>(base + F.counter);
            shape.persistent_groups = F.groups;
            hit_g = reinterpret_cast<uint32_t *>(base + F.hit_g);
            hit_m = reinterpret_cast<uint64_t *>(base + F.hit_m);
        }
    }
    const Layout L = make_layout(scene->n, resolve_leaf(scene->leaf_size));
    T.scenes[0] = make_view(*scene, L);
    T.n_segs = 1;
    T.segs[0].ro = ray_o;
    T.segs[0].rd = ray_d;
    T.segs[0].stride = n_rays;
    T.segs[0].n_rays = n_rays;
    const uint32_t *order = reinterpret_cast<const uint32_t *>(static_cast<const char *>(scene->accel) + L.vals0);
    return map_hip(enqueue_backward(T, A, *scene, order, grad_mean, grad_scale,
                                    grad_quat, grad_density, shape, hit_g, hit_m,
                                    static_cast<hipStream_t>(stream)));
}

// Scratch of gr_project_backward_static: one array per GPU, held until the
// process ends. In host code its name is only a stand-in; the device address
// comes from hipGetSymbolAddress, once per device, and only that address is
// ever handed to kernels.
__device__ __align__(256) unsigned char scratch[GR_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's static scratch (NULL on failure).
void *static_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

gr_status gr_project_backward(const gr_scene *scene, const float *ray_o, const float *ray_d,
                              int64_t n_rays, const float *grad_out, const gr_loss *loss,
                              float *grad_mean, float *grad_scale, float *grad_quat,
                              float *grad_density, void *scratch, size_t scratch_bytes,
                              const gr_launch *opt, void *stream) {
    LaunchShape shape;
    gr_status st = check_launch(opt, shape);
    if (st != GR_OK) return st;
    return backward_common(scene, ray_o, ray_d, n_rays, grad_out, loss, grad_mean, grad_scale, grad_quat,
                           grad_density, scratch, scratch_bytes, shape, opt, stream);
}

gr_status gr_project_backward_static(const gr_scene *scene, const float *ray_o, const float *ray_d,
                                     int64_t n_rays, const float *grad_out, const gr_loss *loss,
                                     float *grad_mean, float *grad_scale, float *grad_quat,
                                     float *grad_density, const gr_launch *opt, void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    size_t acc = 0;
    if ((st = gr_backward_scratch_bytes(scene->n, &acc)) != GR_OK) return st;
    if (acc + 512 > GR_STATIC_SCRATCH_BYTES) return GR_E_UNSUPPORTED;
    LaunchShape shape;
    if ((st = check_launch(opt, shape)) != GR_OK) return st;
    if (!grad_out && shape.hit_cap > 0) {
        // hit lists as long as the rest of the array holds, whole 64-entry
        // batches, else re-traversal
        FusedLayout F;
        LaunchShape none = shape;
        none.hit_cap = 0;
        if ((st = fused_layout(scene->n, opt, none, F)) != GR_OK) return st;
        const size_t waves = size_t(F.groups) * size_t(shape.waves);
        const size_t room = GR_STATIC_SCRATCH_BYTES - F.total - 512;  // two 256-B alignment pads
        size_t cap = room / (waves * (sizeof(uint32_t) + sizeof(uint64_t)));
        cap = (cap / 64) * 64;
        shape.hit_cap = int(cap < size_t(shape.hit_cap) ? cap : size_t(shape.hit_cap));
        if (shape.hit_cap < 64) shape.hit_cap = 0;
    }
    void *ptr = static_scratch();
    if (!ptr) return GR_E_HIP;
    return backward_common(scene, ray_o, ray_d, n_rays, grad_out, loss, grad_mean, grad_scale, grad_quat,
                           grad_density, ptr, GR_STATIC_SCRATCH_BYTES, shape, opt, stream);
}

gr_status gr_backward_accum_zero(int64_t n, float *accum, void *stream) {
    if (n < 0) return GR_E_ARG;
    if (n > GR_MAX_GAUSSIANS) return GR_E_UNSUPPORTED;
    if (n > 0 && (!accum || !aligned(accum, 256))) return GR_E_ARG;
    gr_status st = pending_error();
    if (st != GR_OK) return st;
    enqueue_zero_f32(accum, 10 * n, static_cast<hipStream_t>(stream));
    return map_hip(hipGetLastError());
}

gr_status gr_project_backward_batched(const gr_scene *scenes, int32_t n_scenes, const gr_bwd_segment *segs,
                                      int32_t n_segs, void *scratch, size_t scratch_bytes, const gr_launch *opt,
                                      void *stream) {
    if (!scenes || n_scenes < 1 || n_segs < 0 || (n_segs > 0 && !segs)) return GR_E_ARG;
    if (n_scenes > GR_MAX_SCENES || n_segs > GR_MAX_SEGMENTS) return GR_E_UNSUPPORTED;
    gr_status st;
    for (int s = 0; s < n_scenes; ++s)
        if ((st = check_scene(&scenes[s], true)) != GR_OK) return st;
    for (int k = 0; k < n_segs; ++k) {
        const gr_bwd_segment &g = segs[k];
        if (g.scene < 0 || g.scene >= n_scenes || g.ray_offset < 0 || g.n_rays < 0 ||
            g.out_offset < 0 || g.stride < 0 || g.ray_offset + g.n_rays > g.stride)
            return GR_E_ARG;
        if (g.loss_kind != GR_LOSS_L2 && g.loss_kind != GR_LOSS_POISSON) return GR_E_ARG;
        if (!isfinite(g.background) || (g.loss_kind == GR_LOSS_POISSON && !(g.background > 0.0f)))
            return GR_E_ARG;
        if (g.n_rays > 0 && (!g.ray_o || !g.ray_d || !g.target)) return GR_E_ARG;
        if (scenes[g.scene].n > 0 && (!g.accum || !aligned(g.accum, 256))) return GR_E_ARG;
    }
    LaunchShape shape;
    if ((st = check_launch(opt, shape)) != GR_OK) return st;
    uint32_t *hit_g = nullptr;
    uint64_t *hit_m = nullptr;
    if (scratch) {
        if (!aligned(scratch, 256)) return GR_E_ARG;
        FusedLayout F;
        if ((st = fused_layout(0, opt, shape, F)) != GR_OK) return st;
        if (shape.hit_cap == 0 || scratch_bytes < F.total) return GR_E_WORKSPACE;
        char *base = static_cast<char *>(scratch);
        if (!shape.work_counter) shape.work_counter = reinterpret_cast<uint32_t *>(base + F.counter);
        shape.persistent_groups = F.groups;
        hit_g = reinterpret_cast<uint32_t *>(base + F.hit_g);
        hit_m = reinterpret_cast<uint64_t *>(base + F.hit_m);
    }
    if ((st = pending_error()) != GR_OK) return st;
    LaunchTable T;
    memset(&T, 0, sizeof(T));
    for (int s = 0; s < n_scenes; ++s) {
        const Layout L = make_layout(scenes[s].n, resolve_leaf(scenes[s].leaf_size));
        T.scenes[s] = make_view(scenes[s], L);
    }
    T.n_segs = n_segs;
    for (int k = 0; k < n_segs; ++k) {
        const gr_bwd_segment &g = segs[k];
        Segment &d = T.segs[k];
        d.scene = g.scene;
        d.loss_kind = g.loss_kind;
        d.ro = g.ray_o;
        d.rd = g.ray_d;
        d.stride = g.stride;
        d.ray_offset = g.ray_offset;
        d.n_rays = g.n_rays;
        d.out = g.out_proj;
        d.out_offset = g.out_offset;
        d.target = g.target;
        d.acc = g.accum;
        d.loss = g.out_loss;
        d.background = g.background;
    }
    return map_hip(enqueue_fused_segments(T, shape, hit_g, hit_m, static_cast<hipStream_t>(stream)));
}

gr_status gr_backward_finish(const gr_scene *scene, const float *accum, float *grad_mean, float *grad_scale,
                             float *grad_quat, float *grad_density, void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if (scene->n > 0 && (!accum || !aligned(accum, 256) || !grad_mean || !grad_scale || !grad_quat ||
                         !grad_density))
        return GR_E_ARG;
    if ((st = pending_error()) != GR_OK) return st;
    const Layout L = make_layout(scene->n, resolve_leaf(scene->leaf_size));
    const uint32_t *order = reinterpret_cast<const uint32_t *>(static_cast<const char *>(scene->accel) + L.vals0);
    enqueue_epilogue(*scene, order, accum, grad_mean, grad_scale, grad_quat, grad_density,
                     static_cast<hipStream_t>(stream));
    return map_hip(hipGetLastError());
}

gr_status gr_rays_count_ct(const gr_ct_geom *g, int64_t *n_rays) {
    gr_status st = check_ct(g);
    if (st != GR_OK) return st;
    if (!n_rays) return GR_E_ARG;
    *n_rays = int64_t(g->n_views) * g->nu * g->nv;
    return GR_OK;
}

gr_status gr_rays_count_pet(const gr_pet_geom *g, int64_t *n_rays) {
    int64_t np = 0;
    gr_status st = check_pet(g, np);
    if (st != GR_OK) return st;
    if (!n_rays) return GR_E_ARG;
    *n_rays = int64_t(g->n_views) * g->n_radial * np;
    return GR_OK;
}

gr_status gr_make_rays_ct(const gr_ct_geom *g, float *ray_o, float *ray_d, void *stream) {
    int64_t n = 0;
    gr_status st = gr_rays_count_ct(g, &n);
    if (st != GR_OK) return st;
    if (n > 0 && (!ray_o || !ray_d)) return GR_E_ARG;
    if ((st = pending_error()) != GR_OK) return st;
    return map_hip(enqueue_rays_ct(*g, n, ray_o, ray_d, static_cast<hipStream_t>(stream)));
}

gr_status gr_make_rays_pet_arccorr(const gr_pet_geom *g, float *ray_o, float *ray_d, void *stream) {
    int64_t np = 0;
    gr_status st = check_pet(g, np);
    if (st != GR_OK) return st;
    const int64_t n = int64_t(g->n_views) * g->n_radial * np;
    if (n > 0 && (!ray_o || !ray_d)) return GR_E_ARG;
    if ((st = pending_error()) != GR_OK) return st;
    return map_hip(enqueue_rays_pet(*g, np, n, ray_o, ray_d, static_cast<hipStream_t>(stream)));
}

}  // extern "C"

static gr_status voxelize_impl(const gr_scene *scene, const gr_grid *grid, float *out, uint64_t *stats,
                               void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if (!grid) return GR_E_ARG;
    int64_t total = 1;
    for (int k = 0; k < 3; ++k) {
        if (!isfinite(grid->origin[k]) || !(grid->spacing[k] > 0.0) || !isfinite(grid->spacing[k]))
            return GR_E_ARG;
        if (grid->dims[k] < 0 || grid->dims[k] > (int64_t(1) << 36)) return GR_E_ARG;
    }
    if (grid->dims[0] > 0 && grid->dims[1] > 0 && grid->dims[2] > 0) {
        if (grid->dims[0] * grid->dims[1] > (int64_t(1) << 36) / grid->dims[2]) return GR_E_UNSUPPORTED;
        total = grid->dims[0] * grid->dims[1] * grid->dims[2];
    } else {
        total = 0;
    }
    if (total > 0 && !out) return GR_E_ARG;
    if ((st = pending_error()) != GR_OK) return st;
    if (total == 0) return GR_OK;
    const Layout L = make_layout(scene->n, resolve_leaf(scene->leaf_size));
    return map_hip(enqueue_voxelize(make_view(*scene, L), *grid, out, stats, static_cast<hipStream_t>(stream)));
}

gr_status gr_voxelize(const gr_scene *scene, const gr_grid *grid, float *out, const gr_launch *opt,
                      void *stream) {
    (void)opt;
    return voxelize_impl(scene, grid, out, nullptr, stream);
}

gr_status gr_voxelize_stats(const gr_scene *scene, const gr_grid *grid, float *out, uint64_t *stats,
                            const gr_launch *opt, void *stream) {
    (void)opt;
    if (!stats || !aligned(stats, 8)) return GR_E_ARG;
    return voxelize_impl(scene, grid, out, stats, stream);
}

gr_status gr_adam_step(float *param, const float *grad, float *m, float *v, int64_t count,
                       const gr_adam *hp, void *stream) {
    if (!hp || count < 0) return GR_E_ARG;
    if (count > 0 && (!param || !grad || !m || !v)) return GR_E_ARG;
    if (hp->step < 1 || !(hp->lr >= 0.0f) || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) ||
        !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) || !(hp->eps > 0.0f) || !isfinite(hp->lr))
        return GR_E_ARG;
    gr_status st = pending_error();
    if (st != GR_OK) return st;
    return map_hip(enqueue_adam(param, grad, m, v, count, *hp, static_cast<hipStream_t>(stream)));
}

static bool adam_hp_ok(float lr, float b1, float b2, float eps, int64_t step) {
    return step >= 1 && lr >= 0.0f && isfinite(lr) && b1 >= 0.0f && b1 < 1.0f && b2 >= 0.0f && b2 < 1.0f &&
           eps > 0.0f && isfinite(eps);
}

gr_status gr_adam_gaussians(int64_t n, float *theta, const float *grad, float *m, float *v, float *natural,
                            const gr_gauss_adam *hp, void *stream) {
    if (!hp || n < 0) return GR_E_ARG;
    if (n > (int64_t(1) << 28)) return GR_E_UNSUPPORTED;
    for (int k = 0; k < 4; ++k)
        if (!adam_hp_ok(hp->lr[k], hp->beta1, hp->beta2, hp->eps, hp->step)) return GR_E_ARG;
    if (n > 0) {
        const float *a[5] = {theta, grad, m, v, natural};
        const size_t bytes = size_t(11) * size_t(n) * sizeof(float);
        for (int i = 0; i < 5; ++i) {
            if (!a[i] || !aligned(a[i], 4)) return GR_E_ARG;
            for (int j = 0; j < i; ++j) {
                const char *x = reinterpret_cast<const char *>(a[i]), *y = reinterpret_cast<const char *>(a[j]);
                if (x < y + bytes && y < x + bytes) return GR_E_ARG;
            }
        }
    }
    gr_status st = pending_error();
    if (st != GR_OK) return st;
    return map_hip(enqueue_adam_gaussians(n, theta, grad, m, v, natural, *hp, static_cast<hipStream_t>(stream)));
}

static gr_status check_tof(const gr_tof *tof, int64_t n_rays) {
    if (!tof) return GR_E_ARG;
    if (tof->n_bins < 0) return GR_E_ARG;
    if (tof->n_bins > GR_TOF_MAX_BINS) return GR_E_UNSUPPORTED;
    if (tof->n_bins > 0 && !(tof->sigma > 0.0f && isfinite(tof->sigma) && tof->bin_width > 0.0f &&
                             isfinite(tof->bin_width)))
        return GR_E_ARG;
    if (tof->n_bins > 0 && (tof->sigma < 1e-12f || double(tof->sigma) * double(tof->sigma) > 3e38))
        return GR_E_ARG;
    (void)n_rays;
    return GR_OK;
}

static void tof_table(const gr_scene *scene, const float *ray_o, const float *ray_d, int64_t n_rays,
                      LaunchTable &T, Layout &L) {
    memset(&T, 0, sizeof(T));
    L = make_layout(scene->n, resolve_leaf(scene->leaf_size));
    T.scenes[0] = make_view(*scene, L);
    T.n_segs = 1;
    T.segs[0].ro = ray_o;
    T.segs[0].rd = ray_d;
    T.segs[0].stride = n_rays;
    T.segs[0].n_rays = n_rays;
}

static TofArgs tof_args(const gr_tof *tof, int64_t n_rays) {
    TofArgs A;
    memset(&A, 0, sizeof(A));
    A.n_bins = tof->n_bins;
    A.sigma2 = tof->n_bins > 0 ? tof->sigma * tof->sigma : 0.0f;
    A.width = tof->n_bins > 0 ? tof->bin_width : 0.0f;
    A.center = tof->center;
    A.atten = tof->atten;
    A.n_rays = n_rays;
    return A;
}

gr_status gr_project_tof(const gr_scene *scene, const float *ray_o, const float *ray_d, int64_t n_rays,
                         const gr_tof *tof, float *out, const gr_launch *opt, void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if ((st = check_tof(tof, n_rays)) != GR_OK) return st;
    if (n_rays < 0) return GR_E_ARG;
    if (n_rays > 0 && (!ray_o || !ray_d || !out)) return GR_E_ARG;
    if (n_rays > (int64_t(1) << 40) / (tof->n_bins > 0 ? tof->n_bins : 1)) return GR_E_UNSUPPORTED;
    LaunchShape shape;
    if ((st = check_launch(opt, shape)) != GR_OK) return st;
    if (shape.waves > 4) return GR_E_ARG;  // TOF kernels run at most 4 waves per group
    if ((st = pending_error()) != GR_OK) return st;
    LaunchTable T;
    Layout L;
    tof_table(scene, ray_o, ray_d, n_rays, T, L);
    TofArgs A = tof_args(tof, n_rays);
    A.out = out;
    return map_hip(enqueue_forward_tof(T, A, shape, static_cast<hipStream_t>(stream)));
}

gr_status gr_project_tof_backward(const gr_scene *scene, const float *ray_o, const float *ray_d, int64_t n_rays,
                                  const gr_tof *tof, const float *grad_out, float *grad_mean, float *grad_scale,
                                  float *grad_quat, float *grad_density, void *scratch, size_t scratch_bytes,
                                  const gr_launch *opt, void *stream) {
    gr_status st = check_scene(scene, true);
    if (st != GR_OK) return st;
    if ((st = check_tof(tof, n_rays)) != GR_OK) return st;
    if (n_rays < 0) return GR_E_ARG;
    if (n_rays > 0 && (!ray_o || !ray_d || !grad_out)) return GR_E_ARG;
    if (n_rays > (int64_t(1) << 40) / (tof->n_bins > 0 ? tof->n_bins : 1)) return GR_E_UNSUPPORTED;
    if (scene->n > 0 && (!grad_mean || !grad_scale || !grad_quat || !grad_density)) return GR_E_ARG;
    size_t need = 0;
    gr_backward_scratch_bytes(scene->n, &need);
    if (!scratch || !aligned(scratch, 256)) return GR_E_ARG;
    if (scratch_bytes < need) return GR_E_WORKSPACE;
    LaunchShape shape;
    if ((st = check_launch(opt, shape)) != GR_OK) return st;
    if (shape.waves > 4) return GR_E_ARG;  // TOF kernels run at most 4 waves per group
    if ((st = pending_error()) != GR_OK) return st;
    LaunchTable T;
    Layout L;
    tof_table(scene, ray_o, ray_d, n_rays, T, L);
    TofArgs A = tof_args(tof, n_rays);
    A.grad_out = grad_out;
    A.acc = static_cast<float *>(scratch);
    const uint32_t *order = reinterpret_cast<const uint32_t *>(static_cast<const char *>(scene->accel) + L.vals0);
    return map_hip(enqueue_backward_tof(T, A, *scene, order, grad_mean, grad_scale, grad_quat, grad_density, shape,
                                        static_cast<hipStream_t>(stream)));
}

gr_status gr_tof_centers(const float *ray_o, const float *ray_d, int64_t n_rays, float *center, void *stream) {
    if (n_rays < 0) return GR_E_ARG;
    if (n_rays > 0 && (!ray_o || !ray_d || !center)) return GR_E_ARG;
    gr_status st = pending_error();
    if (st != GR_OK) return st;
    return map_hip(enqueue_tof_centers(ray_o, ray_d, n_rays, center, static_cast<hipStream_t>(stream)));
}

gr_status gr_loss_weights(int32_t kind, const float *proj, const float *target, const float *background,
                          float background_scalar, int64_t count, float *weight, double *loss, void *stream) {
    if (kind != GR_LOSS_L2 && kind != GR_LOSS_POISSON) return GR_E_ARG;
    if (count < 0) return GR_E_ARG;
    if (count > 0 && (!proj || !target || !weight)) return GR_E_ARG;
    if (!isfinite(background_scalar)) return GR_E_ARG;
    if (kind == GR_LOSS_POISSON && !background && !(background_scalar > 0.0f)) return GR_E_ARG;
    if (loss && !aligned(loss, 8)) return GR_E_ARG;
    gr_status st = pending_error();
    if (st != GR_OK) return st;
    return map_hip(enqueue_loss_weights(kind, proj, target, background, background_scalar, count, weight, loss,
                                        static_cast<hipStream_t>(stream)));
}
