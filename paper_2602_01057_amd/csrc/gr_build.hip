// Acceleration-structure build: per-Gaussian preprocessing, Morton codes,
// stable LSD radix sort, Karras radix-tree LBVH over leaves of L Gaussians,
// bottom-up refit. Everything runs on one stream with no host round trip.
//
// Geometry of one Gaussian (Sec. 3.1, Eq. 2): Sigma = R S S^T R^T with R the
// rotation of the unit quaternion and S = diag(s). Its kappa-sigma ellipsoid
// {x : (x-mu)^T Sigma^-1 (x-mu) <= kappa^2} has axis-aligned half extents
// kappa sqrt(Sigma_jj) and support width kappa sqrt(e^T Sigma e) along any e.
#include <float.h>
#include <math.h>

#include "gr_internal.h"

namespace gr {

namespace {

// Margins that keep the FP32 box and slab tests conservative for lines that
// meet the kappa ellipsoid (absolute part in the scene's length unit, mm).
constexpr float kBoxRel = 1.0f / 65536.0f;
constexpr float kBoxAbs = 1e-3f;

__device__ inline bool load_params(const float *__restrict__ mean, const float *__restrict__ scale,
                                   const float *__restrict__ quat, const float *__restrict__ dens,
                                   int64_t n, int64_t i, double mu[3], double s[3], double q[4],
                                   double &rho) {
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
        mu[k] = mean[k * n + i];
        s[k] = scale[k * n + i];
        ok = ok && isfinite(mu[k]) && isfinite(s[k]) && s[k] > 0.0;
    }
    double qq = 0.0;
    for (int k = 0; k < 4; ++k) {
        q[k] = quat[k * n + i];
        ok = ok && isfinite(q[k]);
        qq += q[k] * q[k];
    }
    rho = dens[i];
    ok = ok && isfinite(rho) && qq > 0.0;
    if (ok) {
        const double inv = 1.0 / sqrt(qq);
        for (int k = 0; k < 4; ++k) q[k] *= inv;
    }
    return ok;
}

// Rotation of a unit quaternion (w, v): R = I + 2 w [v]x + 2 [v]x^2, with
// [v]x^2 = v v^T - |v|^2 I. Columns are the local axes in world coordinates.
__device__ inline void rotation(const double q[4], double R[3][3]) {
    const double w = q[0], v[3] = {q[1], q[2], q[3]};
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double cx[3][3] = {{0.0, -v[2], v[1]}, {v[2], 0.0, -v[0]}, {-v[1], v[0], 0.0}};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            R[a][b] = (a == b ? 1.0 - 2.0 * vv : 0.0) + 2.0 * w * cx[a][b] + 2.0 * v[a] * v[b];
}

__device__ inline uint32_t spread10(uint32_t v) {
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

}  // namespace

// ---------------------------------------------------------------------------
// header and bounds
// ---------------------------------------------------------------------------

__global__ void k_build_init(AccelHeader *hdr, int64_t n, int32_t leaf, int32_t n_leaves,
                             float kappa) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    hdr->magic = kMagic;
    hdr->built = 0;
    hdr->n = n;
    hdr->leaf_size = leaf;
    hdr->n_leaves = n_leaves;
    hdr->kappa = kappa;
    hdr->n_invalid = 0;
    for (int k = 0; k < 3; ++k) {
        hdr->bmin[k] = 0xFFFFFFFFu;
        hdr->bmax[k] = 0u;
    }
    for (int k = 0; k < 3; ++k) {
        hdr->root_box[k] = FLT_MAX;
        hdr->root_box[3 + k] = -FLT_MAX;
    }
    hdr->root = n_leaves > 1 ? 0 : ~0;
    hdr->flags = 0;
}

// Refit: keep the Morton order and the tree of the last build, reset what the
// refit recomputes (invalid count, bounds, root box, flags). A workspace that
// was not built for this n and leaf size is flagged; the kernels that follow
// only follow indices they check, so the refit stays memory-safe.
__global__ void k_refit_init(AccelHeader *hdr, int64_t n, int32_t leaf, int32_t n_leaves, float kappa) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t flags = 0;
    if (hdr->magic != kMagic || hdr->built != 1 || hdr->n != n || hdr->leaf_size != leaf ||
        hdr->n_leaves != n_leaves)
        flags = kFlagNotBuilt;
    hdr->magic = kMagic;
    hdr->built = 0;
    hdr->n = n;
    hdr->leaf_size = leaf;
    hdr->n_leaves = n_leaves;
    hdr->kappa = kappa;
    hdr->n_invalid = 0;
    for (int k = 0; k < 3; ++k) {
        hdr->bmin[k] = 0xFFFFFFFFu;
        hdr->bmax[k] = 0u;
    }
    for (int k = 0; k < 3; ++k) {
        hdr->root_box[k] = FLT_MAX;
        hdr->root_box[3 + k] = -FLT_MAX;
    }
    if (flags) hdr->root = n_leaves > 1 ? 0 : ~0;
    hdr->flags = flags;
}

__global__ void k_fill_u32(uint32_t *p, int64_t count, uint32_t v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ __launch_bounds__(256) void k_bounds(const float *__restrict__ mean,
                                                const float *__restrict__ scale,
                                                const float *__restrict__ quat,
                                                const float *__restrict__ dens, int64_t n,
                                                AccelHeader *hdr) {
    __shared__ uint32_t smin[3], smax[3], sbad;
    if (threadIdx.x < 3) {
        smin[threadIdx.x] = 0xFFFFFFFFu;
        smax[threadIdx.x] = 0u;
    }
    if (threadIdx.x == 0) sbad = 0;
    __syncthreads();
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) {
        double mu[3], s[3], q[4], rho;
        if (load_params(mean, scale, quat, dens, n, i, mu, s, q, rho)) {
            for (int k = 0; k < 3; ++k) {
                const uint32_t u = f2ord(float(mu[k]));
                atomicMin(&smin[k], u);
                atomicMax(&smax[k], u);
            }
        } else {
            atomicAdd(&sbad, 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        atomicMin(&hdr->bmin[threadIdx.x], smin[threadIdx.x]);
        atomicMax(&hdr->bmax[threadIdx.x], smax[threadIdx.x]);
    }
    if (threadIdx.x == 0 && sbad) atomicAdd(&hdr->n_invalid, int(sbad));
}

// 30-bit Morton code of the mean inside the valid-mean bounds; invalid
// Gaussians get 0xFFFFFFFF and sort to the end. vals = input index.
__global__ __launch_bounds__(256) void k_morton(const float *__restrict__ mean,
                                                const float *__restrict__ scale,
                                                const float *__restrict__ quat,
                                                const float *__restrict__ dens, int64_t n,
                                                const AccelHeader *__restrict__ hdr,
                                                uint32_t *__restrict__ keys,
                                                uint32_t *__restrict__ vals) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double mu[3], s[3], q[4], rho;
    uint32_t code = 0xFFFFFFFFu;
    if (load_params(mean, scale, quat, dens, n, i, mu, s, q, rho)) {
        code = 0;
        for (int k = 0; k < 3; ++k) {
            float lo = ord2f(hdr->bmin[k]), hi = ord2f(hdr->bmax[k]);
            if (!(hi > lo)) hi = lo + 1.0f;
            float t = (float(mu[k]) - lo) / (hi - lo);
            int c = int(t * 1024.0f);
            c = c < 0 ? 0 : (c > 1023 ? 1023 : c);
            code |= spread10(uint32_t(c)) << (2 - k);
        }
    }
    keys[i] = code;
    vals[i] = uint32_t(i);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits: histogram -> scan -> scatter
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_sort_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                   int shift, uint32_t *__restrict__ hist,
                                                   int nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int k = 0; k < kSortTile / 256; ++k) {
        const int64_t i = base + k * 256 + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[size_t(threadIdx.x) * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of the digit-major histogram (256 x nblocks) in one workgroup.
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t *__restrict__ hist, int m) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (m + 1023) / 1024;
    const int b = t * per, e = min(m, b + per);
    uint32_t s = 0;
    for (int i = b; i < e; ++i) s += hist[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t > 0 ? part[t - 1] : 0u;
    for (int i = b; i < e; ++i) {
        const uint32_t v = hist[i];
        hist[i] = run;
        run += v;
    }
}

// Stable scatter. Each workgroup walks its tile in 16 rounds of 256 keys in
// input order; inside a wave the keys sharing a digit are found with eight
// ballots (one per digit bit), so each key's rank among equal digits is the
// population count of lower lanes with the same digit.
__global__ __launch_bounds__(256) void k_sort_scatter(const uint32_t *__restrict__ kin,
                                                      const uint32_t *__restrict__ vin,
                                                      uint32_t *__restrict__ kout,
                                                      uint32_t *__restrict__ vout, int64_t n,
                                                      int shift, const uint32_t *__restrict__ hist,
                                                      int nblocks) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wsl[4][256];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    run[t] = hist[size_t(t) * nblocks + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int k = 0; k < kSortTile / 256; ++k) {
        const int64_t i = base + k * 256 + t;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t dig = (key >> shift) & 255u;
        for (int ww = 0; ww < 4; ++ww) wsl[ww][t] = 0;
        __syncthreads();
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t bal = __ballot(valid && bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t rank = uint32_t(__popcll(peers & lt));
        if (valid && rank == 0) wsl[w][dig] = uint32_t(__popcll(peers));
        __syncthreads();
        const uint32_t c0 = wsl[0][t], c1 = wsl[1][t], c2 = wsl[2][t], c3 = wsl[3][t];
        const uint32_t g = run[t];
        __syncthreads();
        wsl[0][t] = g;
        wsl[1][t] = g + c0;
        wsl[2][t] = g + c0 + c1;
        wsl[3][t] = g + c0 + c1 + c2;
        run[t] = g + c0 + c1 + c2 + c3;
        __syncthreads();
        if (valid) {
            const uint32_t pos = wsl[w][dig] + rank;
            if (pos < n) {
                kout[pos] = key;
                vout[pos] = val;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// per-Gaussian records in Morton order
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_gather(const float *__restrict__ mean,
                                                const float *__restrict__ scale,
                                                const float *__restrict__ quat,
                                                const float *__restrict__ dens, int64_t n,
                                                float kappa, const uint32_t *__restrict__ order,
                                                GaussRec *__restrict__ rec,
                                                GaussRec32 *__restrict__ rec32,
                                                float *__restrict__ cull,
                                                float *__restrict__ aabb) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int64_t i = order[g];
    double mu[3], s[3], q[4], rho;
    GaussRec r;
    if (i >= n || !load_params(mean, scale, quat, dens, n, i, mu, s, q, rho)) {
        for (int k = 0; k < 3; ++k) r.mu[k] = __builtin_nan("");
        for (int k = 0; k < 6; ++k) r.P[k] = 0.0;
        r.rho_c = 0.0f;
        r.pad = 0.0f;
        rec[g] = r;
        GaussRec32 c;
        for (int k = 0; k < 3; ++k) c.mu[k] = __builtin_nanf("");
        for (int k = 0; k < 9; ++k) c.W[k] = 0.0f;
        c.rho_c = 0.0f;
        c.pad[0] = c.pad[1] = c.pad[2] = 0.0f;
        rec32[g] = c;
        for (int f = 0; f < kCullFields; ++f) cull[f * n + g] = __builtin_nanf("");
        for (int k = 0; k < 3; ++k) {
            aabb[g * 6 + k] = FLT_MAX;
            aabb[g * 6 + 3 + k] = -FLT_MAX;
        }
        return;
    }
    double R[3][3];
    rotation(q, R);
    double Sg[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Sg[a][b] = R[a][0] * R[b][0] * s[0] * s[0] + R[a][1] * R[b][1] * s[1] * s[1] +
                       R[a][2] * R[b][2] * s[2] * s[2];
    // precision matrix P = R diag(s^-2) R^T, the inverse of Sigma
    double Pm[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            Pm[a][b] = R[a][0] * R[b][0] / (s[0] * s[0]) + R[a][1] * R[b][1] / (s[1] * s[1]) +
                       R[a][2] * R[b][2] / (s[2] * s[2]);
    for (int k = 0; k < 3; ++k) r.mu[k] = mu[k];
    r.P[0] = Pm[0][0];
    r.P[1] = Pm[1][1];
    r.P[2] = Pm[2][2];
    r.P[3] = Pm[0][1];
    r.P[4] = Pm[0][2];
    r.P[5] = Pm[1][2];
    r.rho_c = float(rho * 2.5066282746310002);  // rho sqrt(2 pi)
    r.pad = 0.0f;
    rec[g] = r;
    // whitening W = diag(1/s) R^T: row a is the a-th local axis over its scale
    GaussRec32 c;
    for (int k = 0; k < 3; ++k) c.mu[k] = float(mu[k]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) c.W[3 * a + b] = float(R[b][a] / s[a]);
    c.rho_c = r.rho_c;
    c.pad[0] = c.pad[1] = c.pad[2] = 0.0f;
    rec32[g] = c;
    const double k2 = double(kappa) * double(kappa);
    cull[0 * n + g] = float(mu[0]);
    cull[1 * n + g] = float(mu[1]);
    cull[2 * n + g] = float(mu[2]);
    cull[3 * n + g] = float(k2 * Sg[0][0]);
    cull[4 * n + g] = float(k2 * Sg[1][1]);
    cull[5 * n + g] = float(k2 * Sg[2][2]);
    cull[6 * n + g] = float(k2 * Sg[0][1]);
    cull[7 * n + g] = float(k2 * Sg[0][2]);
    cull[8 * n + g] = float(k2 * Sg[1][2]);
    for (int k = 0; k < 3; ++k) {
        const float e = float(double(kappa) * sqrt(Sg[k][k])) * (1.0f + kBoxRel) + kBoxAbs;
        aabb[g * 6 + k] = float(mu[k]) - e;
        aabb[g * 6 + 3 + k] = float(mu[k]) + e;
    }
}

// ---------------------------------------------------------------------------
// Karras radix tree over leaves; leaf l holds Morton positions [l L, (l+1) L)
// ---------------------------------------------------------------------------

__device__ inline int prefix_len(const uint32_t *__restrict__ keys, int leaf, int nl, int i, int j) {
    if (j < 0 || j >= nl) return -1;
    const uint32_t a = keys[size_t(i) * leaf], b = keys[size_t(j) * leaf];
    if (a == b) return 32 + __clz(uint32_t(i ^ j));
    return __clz(a ^ b);
}

__global__ __launch_bounds__(256) void k_karras(const uint32_t *__restrict__ keys, int leaf,
                                                int nl, Node *__restrict__ nodes,
                                                int32_t *__restrict__ lparent, AccelHeader *hdr) {
    const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nl - 1) return;
    const int d = (prefix_len(keys, leaf, nl, i, i + 1) - prefix_len(keys, leaf, nl, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = prefix_len(keys, leaf, nl, i, i - d);
    int lmax = 2;
    while (prefix_len(keys, leaf, nl, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(keys, leaf, nl, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix_len(keys, leaf, nl, i, j);
    int s = 0, step = l;
    do {
        step = (step + 1) >> 1;
        if (prefix_len(keys, leaf, nl, i, i + (s + step) * d) > dnode) s += step;
    } while (step > 1);
    const int gam = i + s * d + (d < 0 ? -1 : 0);
    const int lo = min(i, j), hi = max(i, j);
    const int left = (lo == gam) ? ~gam : gam;
    const int right = (hi == gam + 1) ? ~(gam + 1) : gam + 1;
    const bool ok_l = left < 0 ? (~left < nl) : (left < nl - 1);
    const bool ok_r = right < 0 ? (~right < nl) : (right < nl - 1);
    if (gam < 0 || !ok_l || !ok_r) {
        atomicOr(&hdr->flags, kFlagTreeCorrupt);
        return;
    }
    nodes[i].child[0] = left;
    nodes[i].child[1] = right;
    if (left >= 0) nodes[left].parent = i; else lparent[~left] = i;
    if (right >= 0) nodes[right].parent = i; else lparent[~right] = i;
    if (i == 0) nodes[0].parent = -1;
}

// ---------------------------------------------------------------------------
// bottom-up refit: the second child to finish computes its parent's box
// ---------------------------------------------------------------------------

__device__ inline void leaf_box(const float *__restrict__ aabb, int64_t n, int leaf, int l,
                                float box[6]) {
    for (int k = 0; k < 3; ++k) {
        box[k] = FLT_MAX;
        box[3 + k] = -FLT_MAX;
    }
    const int64_t b = int64_t(l) * leaf, e = min(n, b + leaf);
    for (int64_t g = b; g < e; ++g)
        for (int k = 0; k < 3; ++k) {
            box[k] = fminf(box[k], aabb[g * 6 + k]);
            box[3 + k] = fmaxf(box[3 + k], aabb[g * 6 + 3 + k]);
        }
}

__global__ __launch_bounds__(256) void k_refit(const float *__restrict__ aabb, int64_t n, int leaf,
                                               int nl, Node *nodes,
                                               const int32_t *__restrict__ lparent,
                                               uint32_t *visit, AccelHeader *hdr) {
    const int l = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (l >= nl) return;
    float box[6];
    leaf_box(aabb, n, leaf, l, box);
    const int nn = nl - 1;
    int me = ~l;
    int p = lparent[l];
    // a path to the root has at most nn nodes; the cap only matters if the
    // tree is corrupt
    for (int it = 0; it <= nn; ++it) {
        if (p < 0 || p >= nn) {
            atomicOr(&hdr->flags, kFlagTreeCorrupt);
            return;
        }
        const int slot = (nodes[p].child[0] == me) ? 0 : 1;
        for (int k = 0; k < 6; ++k)
            __hip_atomic_store(&nodes[p].b[6 * slot + k], box[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t old = atomicAdd(&visit[p], 1u);
        if (old == 0) return;
        __threadfence();
        for (int k = 0; k < 3; ++k) {
            const float a0 = __hip_atomic_load(&nodes[p].b[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const float a1 = __hip_atomic_load(&nodes[p].b[6 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const float c0 = __hip_atomic_load(&nodes[p].b[3 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const float c1 = __hip_atomic_load(&nodes[p].b[9 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            box[k] = fminf(a0, a1);
            box[3 + k] = fmaxf(c0, c1);
        }
        me = p;
        p = nodes[p].parent;
        if (p == -1 && me == 0) {
            for (int k = 0; k < 6; ++k) hdr->root_box[k] = box[k];
            return;
        }
    }
    atomicOr(&hdr->flags, kFlagTreeCorrupt);
}

// One leaf (n <= L): the root is that leaf.
__global__ void k_single_leaf(const float *__restrict__ aabb, int64_t n, int leaf,
                              AccelHeader *hdr) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float box[6];
    leaf_box(aabb, n, leaf, 0, box);
    for (int k = 0; k < 6; ++k) hdr->root_box[k] = box[k];
}

// Wide hierarchy, level 0: one box per leaf (union of its Gaussians).
__global__ __launch_bounds__(256) void k_wide_leaves(const float *__restrict__ aabb, int64_t n,
                                                     int leaf, int nl, float *__restrict__ wbox,
                                                     int total) {
    const int l = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (l >= nl) return;
    float box[6];
    leaf_box(aabb, n, leaf, l, box);
    for (int k = 0; k < 6; ++k) wbox[size_t(k) * total + l] = box[k];
}

// Wide hierarchy, level > 0: node i is the union of children [64 i, 64 i + 64)
// of the level below.
__global__ __launch_bounds__(256) void k_wide_level(float *__restrict__ wbox, int total, int child_off,
                                                    int child_count, int off, int count) {
    const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float box[6];
    for (int k = 0; k < 3; ++k) {
        box[k] = FLT_MAX;
        box[3 + k] = -FLT_MAX;
    }
    const int c0 = i * kWide, c1 = min(child_count, c0 + kWide);
    for (int c = c0; c < c1; ++c)
        for (int k = 0; k < 3; ++k) {
            box[k] = fminf(box[k], wbox[size_t(k) * total + child_off + c]);
            box[3 + k] = fmaxf(box[3 + k], wbox[size_t(3 + k) * total + child_off + c]);
        }
    for (int k = 0; k < 6; ++k) wbox[size_t(k) * total + off + i] = box[k];
}

__global__ void k_build_done(AccelHeader *hdr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) hdr->built = 1;
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(int64_t count, int threads) {
    return unsigned((count + threads - 1) / threads);
}

// Node boxes of the binary tree (bottom-up from the leaves) and the wide
// hierarchy, from the per-Gaussian boxes in Morton order.
static void enqueue_boxes(const gr_scene &sc, const Layout &L, char *base, AccelHeader *hdr, hipStream_t st) {
    const int64_t n = sc.n;
    float *aabb = reinterpret_cast<float *>(base + L.aabb);
    if (L.n_leaves > 1) {
        Node *nodes = reinterpret_cast<Node *>(base + L.nodes);
        int32_t *lpar = reinterpret_cast<int32_t *>(base + L.lparent);
        uint32_t *visit = reinterpret_cast<uint32_t *>(base + L.visit);
        k_fill_u32<<<blocks_for(L.n_nodes, 256), 256, 0, st>>>(visit, L.n_nodes, 0u);
        k_refit<<<blocks_for(L.n_leaves, 256), 256, 0, st>>>(aabb, n, L.leaf, L.n_leaves, nodes, lpar, visit,
                                                             hdr);
    } else {
        k_single_leaf<<<1, 64, 0, st>>>(aabb, n, L.leaf, hdr);
    }
    float *wbox = reinterpret_cast<float *>(base + L.wbox);
    k_wide_leaves<<<blocks_for(L.n_leaves, 256), 256, 0, st>>>(aabb, n, L.leaf, L.n_leaves, wbox, L.wide_total);
    for (int lv = 1; lv < L.n_levels; ++lv)
        k_wide_level<<<blocks_for(L.level_count[lv], 256), 256, 0, st>>>(
            wbox, L.wide_total, L.level_off[lv - 1], L.level_count[lv - 1], L.level_off[lv], L.level_count[lv]);
}

hipError_t enqueue_refit(const gr_scene &sc, const Layout &L, hipStream_t st) {
    char *base = static_cast<char *>(sc.accel);
    AccelHeader *hdr = reinterpret_cast<AccelHeader *>(base);
    const int64_t n = sc.n;
    k_refit_init<<<1, 64, 0, st>>>(hdr, n, L.leaf, L.n_leaves, sc.kappa);
    if (n > 0) {
        const uint32_t *order = reinterpret_cast<const uint32_t *>(base + L.vals0);
        k_bounds<<<blocks_for(n, 256), 256, 0, st>>>(sc.mean, sc.scale, sc.quat, sc.density, n, hdr);
        k_gather<<<blocks_for(n, 256), 256, 0, st>>>(sc.mean, sc.scale, sc.quat, sc.density, n, sc.kappa, order,
                                                      reinterpret_cast<GaussRec *>(base + L.rec),
                                                      reinterpret_cast<GaussRec32 *>(base + L.rec32),
                                                      reinterpret_cast<float *>(base + L.cull),
                                                      reinterpret_cast<float *>(base + L.aabb));
        enqueue_boxes(sc, L, base, hdr, st);
    }
    k_build_done<<<1, 64, 0, st>>>(hdr);
    return hipGetLastError();
}

hipError_t enqueue_build(const gr_scene &sc, const Layout &L, hipStream_t st) {
    char *base = static_cast<char *>(sc.accel);
    AccelHeader *hdr = reinterpret_cast<AccelHeader *>(base);
    const int64_t n = sc.n;
    k_build_init<<<1, 64, 0, st>>>(hdr, n, L.leaf, L.n_leaves, sc.kappa);
    if (n > 0) {
        uint32_t *k0 = reinterpret_cast<uint32_t *>(base + L.keys0);
        uint32_t *k1 = reinterpret_cast<uint32_t *>(base + L.keys1);
        uint32_t *v0 = reinterpret_cast<uint32_t *>(base + L.vals0);
        uint32_t *v1 = reinterpret_cast<uint32_t *>(base + L.vals1);
        uint32_t *hist = reinterpret_cast<uint32_t *>(base + L.hist);
        k_bounds<<<blocks_for(n, 256), 256, 0, st>>>(sc.mean, sc.scale, sc.quat, sc.density, n, hdr);
        k_morton<<<blocks_for(n, 256), 256, 0, st>>>(sc.mean, sc.scale, sc.quat, sc.density, n, hdr,
                                                      k0, v0);
        const int nb = L.n_sort_blocks;
        uint32_t *kin = k0, *vin = v0, *kout = k1, *vout = v1;
        for (int pass = 0; pass < 4; ++pass) {
            const int shift = 8 * pass;
            k_sort_hist<<<nb, 256, 0, st>>>(kin, n, shift, hist, nb);
            k_sort_scan<<<1, 1024, 0, st>>>(hist, 256 * nb);
            k_sort_scatter<<<nb, 256, 0, st>>>(kin, vin, kout, vout, n, shift, hist, nb);
            uint32_t *tk = kin, *tv = vin;
            kin = kout;
            vin = vout;
            kout = tk;
            vout = tv;
        }
        // four passes: the sorted keys and order are back in keys0 / vals0
        GaussRec *rec = reinterpret_cast<GaussRec *>(base + L.rec);
        float *cull = reinterpret_cast<float *>(base + L.cull);
        float *aabb = reinterpret_cast<float *>(base + L.aabb);
        GaussRec32 *rec32 = reinterpret_cast<GaussRec32 *>(base + L.rec32);
        k_gather<<<blocks_for(n, 256), 256, 0, st>>>(sc.mean, sc.scale, sc.quat, sc.density, n,
                                                      sc.kappa, v0, rec, rec32, cull, aabb);
        if (L.n_leaves > 1) {
            Node *nodes = reinterpret_cast<Node *>(base + L.nodes);
            int32_t *lpar = reinterpret_cast<int32_t *>(base + L.lparent);
            uint32_t *visit = reinterpret_cast<uint32_t *>(base + L.visit);
            k_fill_u32<<<blocks_for(L.n_nodes, 256), 256, 0, st>>>(visit, L.n_nodes, 0u);
            k_fill_u32<<<blocks_for(L.n_leaves, 256), 256, 0, st>>>(reinterpret_cast<uint32_t *>(lpar),
                                                                     L.n_leaves, 0xFFFFFFFFu);
            k_karras<<<blocks_for(L.n_nodes, 256), 256, 0, st>>>(k0, L.leaf, L.n_leaves, nodes, lpar, hdr);
            k_refit<<<blocks_for(L.n_leaves, 256), 256, 0, st>>>(aabb, n, L.leaf, L.n_leaves, nodes,
                                                                 lpar, visit, hdr);
        } else {
            float *aabb2 = aabb;
            k_single_leaf<<<1, 64, 0, st>>>(aabb2, n, L.leaf, hdr);
        }
    }
    if (n > 0) {
        // wide hierarchy over the Morton-ordered leaves
        const float *aabb = reinterpret_cast<const float *>(base + L.aabb);
        float *wbox = reinterpret_cast<float *>(base + L.wbox);
        k_wide_leaves<<<blocks_for(L.n_leaves, 256), 256, 0, st>>>(aabb, n, L.leaf, L.n_leaves, wbox,
                                                                   L.wide_total);
        for (int lv = 1; lv < L.n_levels; ++lv)
            k_wide_level<<<blocks_for(L.level_count[lv], 256), 256, 0, st>>>(
                wbox, L.wide_total, L.level_off[lv - 1], L.level_count[lv - 1], L.level_off[lv],
                L.level_count[lv]);
    }
    k_build_done<<<1, 64, 0, st>>>(hdr);
    return hipGetLastError();
}

}  // namespace gr
