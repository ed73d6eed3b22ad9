// Reconstruction-loop kernels: voxelisation of the Gaussian mixture (the
// reconstruction is the optimised Gaussians voxelised, Fig. 1; the field is
// Eq. 2's sum of Gaussians with the projection's kappa cutoff) and one Adam
// step on a parameter array (the optimiser of Sec. 4.1).
#include "gr_internal.h"

namespace gr {

namespace {

constexpr float kInvSqrt2Pi = 0.39894228040143268f;
constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2
constexpr float kBoxPad = 1e-3f;                   // mm added to the brick box

// Grid of voxel centres: origin + (ix, iy, iz) * spacing, x fastest.
struct VoxGrid {
    double origin[3];
    double spacing[3];
    int64_t dims[3];
    int64_t bricks[3];  // bricks per axis
};

// Bricks of kBrick x kBrick x kBrickZ voxels: one wave each, lane (lx, ly) =
// (lane % 8, lane / 8) holding the column of kBrickZ voxels along z.
constexpr int kBrick = 8;
constexpr int kBrickZ = 8;

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

template <class T>
using const_ptr = const __attribute__((address_space(4))) T *;
template <class T>
__device__ inline T sload(const T *p, int64_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const_ptr<T>)p)[i];
#else
    return p[i];
#endif
}

__device__ inline bool boxes_meet(const float lo[3], const float hi[3], const float blo[3],
                                  const float bhi[3]) {
    return lo[0] <= bhi[0] && hi[0] >= blo[0] && lo[1] <= bhi[1] && hi[1] >= blo[1] && lo[2] <= bhi[2] &&
           hi[2] >= blo[2];
}

// Node count and offset of level lv of the wide hierarchy (level 0 = leaves).
__device__ inline void level_info(int n_leaves, int lv, int &cnt, int &off) {
    cnt = n_leaves;
    off = 0;
    for (int k = 0; k < lv; ++k) {
        off += cnt;
        cnt = (cnt + kWide - 1) / kWide;
    }
}

constexpr int kStack = 64 * (kMaxLevels - 1);

// One wave per brick of 8x8x8 voxels, each lane a column of 8 voxels along
// z. The wide hierarchy is walked with box-versus-brick tests, 64 child boxes
// per wave step; at a leaf the Gaussians are culled lane-parallel against the
// brick, and the candidates' records (scalar loads) are evaluated at every
// voxel: D = (x - mu)^T P (x - mu) in FP64 (along the column D is a quadratic
// in z: D(t) = D0 + t (2 h (P delta0)_z) + t^2 h^2 P_zz), rho exp(-D/2) in
// FP32, summed in FP64. With kStats, stats[0] += (voxel, Gaussian) pairs with
// D <= kappa^2 and stats[1] += pairs evaluated (candidates x valid voxels).
template <bool kStats>
__global__ __launch_bounds__(256) void k_voxelize(SceneView S, VoxGrid G, float *__restrict__ out,
                                                 uint64_t *__restrict__ stats) {
    __shared__ uint32_t stack_all[4][kStack];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    uint32_t *stack = stack_all[wave];
    const int64_t brick = int64_t(blockIdx.x) * 4 + wave;
    const int64_t nbx = G.bricks[0], nby = G.bricks[1], nbz = G.bricks[2];
    if (brick >= nbx * nby * nbz) return;
    const int64_t bx = brick % nbx, by = (brick / nbx) % nby, bz = brick / (nbx * nby);
    const int64_t ix = bx * kBrick + (lane & 7), iy = by * kBrick + (lane >> 3), iz0 = bz * kBrickZ;
    const bool xy_valid = ix < G.dims[0] && iy < G.dims[1];
    const int nzv = int(G.dims[2] - iz0 < kBrickZ ? G.dims[2] - iz0 : kBrickZ);  // valid z in the brick
    const double x[3] = {G.origin[0] + double(ix) * G.spacing[0], G.origin[1] + double(iy) * G.spacing[1],
                         G.origin[2] + double(iz0) * G.spacing[2]};
    const double hz = G.spacing[2];
    // the brick's box (its valid voxels), padded
    float blo[3], bhi[3];
    {
        const int64_t i0[3] = {bx * kBrick, by * kBrick, iz0};
        for (int k = 0; k < 3; ++k) {
            const int64_t e = k == 2 ? kBrickZ : kBrick;
            const int64_t i1 = (i0[k] + e - 1 < G.dims[k] ? i0[k] + e - 1 : G.dims[k] - 1);
            const double a = G.origin[k] + double(i0[k]) * G.spacing[k];
            const double b = G.origin[k] + double(i1) * G.spacing[k];
            blo[k] = float(a) - kBoxPad - 1e-6f * fabsf(float(a));
            bhi[k] = float(b) + kBoxPad + 1e-6f * fabsf(float(b));
        }
    }
    const float k2 = S.kappa2;
    const float kap = sqrtf(k2);
    double bc[3];
    float be[3];
    for (int k = 0; k < 3; ++k) {
        bc[k] = 0.5 * (double(blo[k]) + double(bhi[k]));
        be[k] = 0.5f * (bhi[k] - blo[k]) * 1.0001f;
    }
    double acc[kBrickZ];
    for (int t = 0; t < kBrickZ; ++t) acc[t] = 0.0;
    int32_t err = 0;
    uint32_t n_in = 0, n_eval = 0;
    const int top = S.n_levels - 1;
    int n_top, top_off;
    level_info(S.n_leaves, top, n_top, top_off);
    int sp = 0, next_root = 0;
    while (true) {
        int lv, first, cnt, off;
        if (sp > 0) {
            --sp;
            const uint32_t e = uint32_t(__builtin_amdgcn_readfirstlane(int(stack[sp])));
            lv = int(e >> 28) - 1;
            first = int(e & 0x0FFFFFFFu) * kWide;
            int lc;
            level_info(S.n_leaves, lv, lc, off);
            cnt = min(kWide, lc - first);
        } else if (next_root < n_top) {
            lv = top;
            off = top_off;
            first = next_root;
            cnt = min(kWide, n_top - next_root);
            next_root += kWide;
        } else {
            break;
        }
        bool hit = false;
        if (lane < cnt) {
            const int64_t i = int64_t(off) + first + lane;
            const int64_t t = S.wide_total;
            const float lo[3] = {S.wbox[i], S.wbox[t + i], S.wbox[2 * t + i]};
            const float hi[3] = {S.wbox[3 * t + i], S.wbox[4 * t + i], S.wbox[5 * t + i]};
            hit = boxes_meet(lo, hi, blo, bhi);
        }
        uint64_t mask = ballot(hit);
        if (lv == 0) {
            while (mask) {
                const int leaf = first + __builtin_ctzll(mask);
                mask &= mask - 1;
                // the leaf's Gaussians whose kappa-ellipsoid may meet the brick:
                // their kappa-box meets it, and no separating axis along the
                // ellipsoid's normal at the brick centre, u = P (c - mu): the
                // ellipsoid spans u.mu +- kappa sqrt(D(c)) on it, the brick
                // u.c +- sum |u_k| e_k, and u.(c - mu) = D(c)
                const int64_t start = int64_t(leaf) * S.leaf;
                const int64_t rem = S.n - start;
                const int gc = rem < S.leaf ? int(rem) : S.leaf;
                bool cand = false;
                if (lane < gc) {
                    const int64_t g = start + lane;
                    const float mu[3] = {S.cull[g], S.cull[S.n + g], S.cull[2 * S.n + g]};
                    const float h[3] = {sqrtf(fmaxf(S.cull[3 * S.n + g], 0.0f)),
                                        sqrtf(fmaxf(S.cull[4 * S.n + g], 0.0f)),
                                        sqrtf(fmaxf(S.cull[5 * S.n + g], 0.0f))};
                    float lo[3], hi[3];
                    for (int k = 0; k < 3; ++k) {
                        lo[k] = mu[k] - h[k];
                        hi[k] = mu[k] + h[k];
                    }
                    cand = boxes_meet(lo, hi, blo, bhi);
                    if (cand) {
                        const GaussRec &R = S.rec[g];
                        float dl[3], P[6];
                        for (int k = 0; k < 3; ++k) dl[k] = float(bc[k] - R.mu[k]);
                        for (int k = 0; k < 6; ++k) P[k] = float(R.P[k]);
                        const float u[3] = {P[0] * dl[0] + P[3] * dl[1] + P[4] * dl[2],
                                            P[3] * dl[0] + P[1] * dl[1] + P[5] * dl[2],
                                            P[4] * dl[0] + P[5] * dl[1] + P[2] * dl[2]};
                        const float D = u[0] * dl[0] + u[1] * dl[1] + u[2] * dl[2];
                        // |u|.|dl|: scale of the rounding error of D in FP32
                        const float Dabs = fabsf(u[0] * dl[0]) + fabsf(u[1] * dl[1]) + fabsf(u[2] * dl[2]);
                        const float reach = fabsf(u[0]) * be[0] + fabsf(u[1]) * be[1] + fabsf(u[2]) * be[2];
                        if (D > k2) {
                            const float sd = sqrtf(D);
                            if (sd * (sd - kap) > 1.001f * reach + 1e-3f * Dabs + 1e-3f) cand = false;
                        }
                    }
                }
                uint64_t cm = ballot(cand);
                auto eval = [&](const GaussRec &R) {
                    const double dx = x[0] - R.mu[0], dy = x[1] - R.mu[1], dz = x[2] - R.mu[2];
                    const double cx = fma(R.P[4], dz, fma(R.P[3], dy, R.P[0] * dx));
                    const double cy = fma(R.P[5], dz, fma(R.P[1], dy, R.P[3] * dx));
                    const double cz = fma(R.P[2], dz, fma(R.P[5], dy, R.P[4] * dx));
                    const double D0 = fma(dz, cz, fma(dy, cy, dx * cx));
                    const double b1 = 2.0 * hz * cz, c2 = hz * hz * R.P[2];
                    const float w = R.rho_c * kInvSqrt2Pi;
#pragma unroll
                    for (int t = 0; t < kBrickZ; ++t) {
                        const double tt = double(t);
                        const float Df = float(fma(fma(c2, tt, b1), tt, D0));
                        const bool in = Df <= k2;
                        const float e = w * __builtin_amdgcn_exp2f(-kHalfLog2e * Df);
                        acc[t] += in ? double(e) : 0.0;
                        if (kStats) {
                            const bool v = xy_valid && t < nzv;
                            n_eval += v;
                            n_in += v && in;
                        }
                    }
                };
                // two records per step: both scalar loads are in flight at once
                while (cm) {
                    const int j0 = __builtin_ctzll(cm);
                    cm &= cm - 1;
                    const GaussRec R0 = sload(S.rec, start + j0);
                    if (cm) {
                        const int j1 = __builtin_ctzll(cm);
                        cm &= cm - 1;
                        const GaussRec R1 = sload(S.rec, start + j1);
                        eval(R0);
                        eval(R1);
                    } else {
                        eval(R0);
                    }
                }
            }
        } else {
            const int nh = __builtin_popcountll(mask);
            if (sp + nh > kStack) {
                err |= 2;
                continue;
            }
            if ((mask >> lane) & 1ull) {
                const int above = __builtin_popcountll(mask >> lane) - 1;
                stack[sp + above] = (uint32_t(lv) << 28) | uint32_t(first + lane);
            }
            __builtin_amdgcn_wave_barrier();
            sp += nh;
        }
    }
    if (err && lane == 0) atomicOr(const_cast<int32_t *>(&S.hdr->flags), err);
    if (xy_valid)
        for (int t = 0; t < nzv; ++t) out[((iz0 + t) * G.dims[1] + iy) * G.dims[0] + ix] = float(acc[t]);
    if (kStats) {
        uint64_t a = n_in, b = n_eval;
        for (int o = 32; o > 0; o >>= 1) {
            a += __shfl_xor(a, o);
            b += __shfl_xor(b, o);
        }
        if (lane == 0) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&stats[0]), (unsigned long long)a);
            atomicAdd(reinterpret_cast<unsigned long long *>(&stats[1]), (unsigned long long)b);
        }
    }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t count, float lr, float b1, float b2, float eps,
                       float inv_c1, float inv_c2) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * inv_c1) / (sqrtf(vi * inv_c2) + eps);
}

// Per-group constants of the fused step: the rows of a Gaussian scene are
// mean (0-2), log-scale (3-5), quaternion (6-9) and log-density (10).
struct GaussAdamArgs {
    float lr[4];
    float b1, b2, eps, inv_c1, inv_c2;
};

__device__ inline int row_group(int row) { return row < 3 ? 0 : row < 6 ? 1 : row < 10 ? 2 : 3; }

// One thread per (row, Gaussian); blockIdx.y is the row, so the group, its
// learning rate and whether the row is a logarithm are uniform per block.
// Log rows take dL/dlog(x) = dL/dx * x with x the value the projector used.
__global__ __launch_bounds__(256) void k_adam_gaussians(int64_t n, float *__restrict__ theta,
                                                        const float *__restrict__ grad, float *__restrict__ m,
                                                        float *__restrict__ v, float *__restrict__ natural,
                                                        GaussAdamArgs a) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int row = blockIdx.y;
    const int grp = row_group(row);
    const bool is_log = grp == 1 || grp == 3;
    const int64_t k = int64_t(row) * n + i;
    float g = grad[k];
    if (is_log) g *= natural[k];
    const float mi = fmaf(a.b1, m[k], (1.0f - a.b1) * g);
    const float vi = fmaf(a.b2, v[k], (1.0f - a.b2) * g * g);
    m[k] = mi;
    v[k] = vi;
    const float t = theta[k] - a.lr[grp] * (mi * a.inv_c1) / (sqrtf(vi * a.inv_c2) + a.eps);
    theta[k] = t;
    natural[k] = is_log ? expf(t) : t;
}

}  // namespace

hipError_t enqueue_voxelize(const SceneView &S, const gr_grid &g, float *out, uint64_t *stats,
                            hipStream_t st) {
    VoxGrid G;
    for (int k = 0; k < 3; ++k) {
        G.origin[k] = g.origin[k];
        G.spacing[k] = g.spacing[k];
        G.dims[k] = g.dims[k];
        G.bricks[k] = (g.dims[k] + (k == 2 ? kBrickZ : kBrick) - 1) / (k == 2 ? kBrickZ : kBrick);
    }
    const int64_t bricks = G.bricks[0] * G.bricks[1] * G.bricks[2];
    if (bricks == 0) return hipSuccess;
    if (stats)
        k_voxelize<true><<<unsigned((bricks + 3) / 4), 256, 0, st>>>(S, G, out, stats);
    else
        k_voxelize<false><<<unsigned((bricks + 3) / 4), 256, 0, st>>>(S, G, out, nullptr);
    return hipGetLastError();
}

hipError_t enqueue_adam(float *p, const float *g, float *m, float *v, int64_t count, const gr_adam &hp,
                        hipStream_t st) {
    if (count == 0) return hipSuccess;
    const double c1 = 1.0 - pow(double(hp.beta1), double(hp.step));
    const double c2 = 1.0 - pow(double(hp.beta2), double(hp.step));
    k_adam<<<unsigned((count + 255) / 256), 256, 0, st>>>(p, g, m, v, count, hp.lr, hp.beta1, hp.beta2, hp.eps,
                                                          float(1.0 / c1), float(1.0 / c2));
    return hipGetLastError();
}

hipError_t enqueue_adam_gaussians(int64_t n, float *theta, const float *grad, float *m, float *v, float *natural,
                                  const gr_gauss_adam &hp, hipStream_t st) {
    if (n == 0) return hipSuccess;
    GaussAdamArgs a;
    for (int k = 0; k < 4; ++k) a.lr[k] = hp.lr[k];
    a.b1 = hp.beta1;
    a.b2 = hp.beta2;
    a.eps = hp.eps;
    a.inv_c1 = float(1.0 / (1.0 - pow(double(hp.beta1), double(hp.step))));
    a.inv_c2 = float(1.0 / (1.0 - pow(double(hp.beta2), double(hp.step))));
    const dim3 grid(unsigned((n + 255) / 256), 11);
    k_adam_gaussians<<<grid, 256, 0, st>>>(n, theta, grad, m, v, natural, a);
    return hipGetLastError();
}

}  // namespace gr
