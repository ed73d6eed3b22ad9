// Internal device-side layouts and helpers of libgr (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gr.h"

namespace gr {

constexpr uint32_t kMagic = 0x47524143u;  // "GRAC"
constexpr int kDefaultLeaf = 64;
constexpr int kDefaultHitCap = 8192;  // hit-list entries per wave (fused backward)
constexpr int kSortTile = 4096;  // keys per radix-sort workgroup (256 threads x 16)
constexpr int kCullFields = 9;   // mean (3) + kappa^2 Sigma (6: xx yy zz xy xz yz)

// Gaussian record, one per Gaussian in Morton order (80 bytes; a wave
// fetches it with two scalar loads):
//   mu   : the FP32 mean widened to FP64 (exact)
//   P    : Sigma^-1 = R diag(s^-2) R^T in FP64, order xx yy zz xy xz yz
//   rho_c: rho * sqrt(2 pi)
struct alignas(16) GaussRec {
    double mu[3];
    double P[6];
    float rho_c;
    float pad;
};
static_assert(sizeof(GaussRec) == 80, "GaussRec must be 80 bytes");

// Compact FP32 record of the same Gaussian (64 bytes, one scalar load), for
// the forward's FP32 precision mode:
//   mu   : the FP32 mean
//   W    : the whitening matrix diag(1/s) R^T, row-major (P = W^T W)
//   rho_c: rho * sqrt(2 pi)
struct alignas(16) GaussRec32 {
    float mu[3];
    float W[9];
    float rho_c;
    float pad[3];
};
static_assert(sizeof(GaussRec32) == 64, "GaussRec32 must be 64 bytes");

// Binary LBVH internal node with both child boxes inline (64 bytes, one
// scalar load). Box layout: min x, y, z, max x, y, z. child >= 0 is an
// internal node, child < 0 is leaf ~child. An empty child box has min > max.
struct alignas(64) Node {
    float b[12];
    int32_t child[2];
    int32_t parent;
    int32_t pad;
};
static_assert(sizeof(Node) == 64, "Node must be 64 bytes");

// Header at offset 0 of the acceleration workspace.
struct alignas(256) AccelHeader {
    uint32_t magic;
    int32_t built;
    int64_t n;
    int32_t leaf_size;
    int32_t n_leaves;
    float kappa;
    int32_t n_invalid;
    uint32_t bmin[3];  // order-preserving uint encodings of the valid-mean bounds
    uint32_t bmax[3];
    float root_box[6];
    int32_t root;      // internal node index, or ~leaf when there is one leaf
    int32_t flags;
};

constexpr int kWide = 64;      // children per node of the wide hierarchy
constexpr int kMaxLevels = 6;  // leaves + up to 5 wide levels (64^5 leaves)

struct Layout {
    int64_t n;
    int32_t leaf;
    int32_t n_leaves;
    int32_t n_nodes;
    int32_t n_sort_blocks;
    // wide hierarchy: level 0 = leaves, level l has ceil(count[l-1] / 64) nodes,
    // the top level has one node; boxes SoA (6 arrays of wide_total floats)
    int32_t n_levels;
    int32_t level_count[kMaxLevels];
    int32_t level_off[kMaxLevels];
    int32_t wide_total;
    size_t rec, rec32, cull, nodes, aabb, keys0, keys1, vals0, vals1, hist, lparent, visit, wbox, total;
};

__device__ __host__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline Layout make_layout(int64_t n, int32_t leaf) {
    Layout L{};
    L.n = n;
    L.leaf = leaf;
    L.n_leaves = n > 0 ? int32_t((n + leaf - 1) / leaf) : 1;
    L.n_nodes = L.n_leaves > 1 ? L.n_leaves - 1 : 0;
    L.n_sort_blocks = n > 0 ? int32_t((n + kSortTile - 1) / kSortTile) : 1;
    const size_t nn = size_t(n > 0 ? n : 1);
    const size_t nodes = size_t(L.n_nodes > 0 ? L.n_nodes : 1);
    size_t off = align256(sizeof(AccelHeader));
    L.rec = off;     off = align256(off + nn * sizeof(GaussRec));
    L.rec32 = off;   off = align256(off + nn * sizeof(GaussRec32));
    L.cull = off;    off = align256(off + nn * kCullFields * sizeof(float));
    L.nodes = off;   off = align256(off + nodes * sizeof(Node));
    L.aabb = off;    off = align256(off + nn * 6 * sizeof(float));
    L.keys0 = off;   off = align256(off + nn * 4);
    L.keys1 = off;   off = align256(off + nn * 4);
    L.vals0 = off;   off = align256(off + nn * 4);   // after sorting: Morton order -> input index
    L.vals1 = off;   off = align256(off + nn * 4);
    L.hist = off;    off = align256(off + size_t(256) * L.n_sort_blocks * 4);
    L.lparent = off; off = align256(off + size_t(L.n_leaves) * 4);
    L.visit = off;   off = align256(off + nodes * 4);
    int32_t cnt = L.n_leaves, tot = 0, lv = 0;
    while (true) {
        L.level_count[lv] = cnt;
        L.level_off[lv] = tot;
        tot += cnt;
        ++lv;
        if (cnt == 1 || lv == kMaxLevels) break;
        cnt = (cnt + kWide - 1) / kWide;
    }
    L.n_levels = lv;
    L.wide_total = tot;
    L.wbox = off;    off = align256(off + size_t(6) * size_t(tot) * sizeof(float));
    L.total = off;
    return L;
}

// Device view of one built scene, passed by value to the projection kernels.
struct SceneView {
    const AccelHeader *hdr;
    const GaussRec *rec;
    const float *cull;  // kCullFields SoA arrays of length n
    const Node *nodes;
    const uint32_t *order;  // Morton position -> input index
    int64_t n;
    int32_t leaf;
    float kappa2;
    int32_t n_leaves;
    int32_t n_nodes;
    const float *wbox;      // 6 SoA arrays (min xyz, max xyz) of wide_total boxes
    int32_t wide_total;
    int32_t n_levels;  // level k has ceil(n_leaves / 64^k) nodes
};

// The compact records follow the FP64 records in the workspace (make_layout);
// their address is derived here rather than passed, which keeps the launch
// table within the kernel-argument limit.
__device__ __host__ inline const GaussRec32 *rec32_of(const SceneView &v) {
    const size_t nn = size_t(v.n > 0 ? v.n : 1);
    return reinterpret_cast<const GaussRec32 *>(reinterpret_cast<const char *>(v.rec) +
                                                align256(nn * sizeof(GaussRec)));
}

// Error bits recorded in AccelHeader::flags by defensive device-side checks.
enum : int32_t { kFlagTreeCorrupt = 1, kFlagStackOverflow = 2, kFlagTraversalCap = 4, kFlagNotBuilt = 8 };

inline SceneView make_view(const gr_scene &s, const Layout &L) {
    const char *base = static_cast<const char *>(s.accel);
    SceneView v;
    v.hdr = reinterpret_cast<const AccelHeader *>(base);
    v.rec = reinterpret_cast<const GaussRec *>(base + L.rec);
    v.cull = reinterpret_cast<const float *>(base + L.cull);
    v.nodes = reinterpret_cast<const Node *>(base + L.nodes);
    v.order = reinterpret_cast<const uint32_t *>(base + L.vals0);
    v.n = s.n;
    v.leaf = L.leaf;
    v.kappa2 = s.kappa * s.kappa;
    v.n_leaves = L.n_leaves;
    v.n_nodes = L.n_nodes;
    v.wbox = reinterpret_cast<const float *>(base + L.wbox);
    v.wide_total = L.wide_total;
    v.n_levels = L.n_levels;
    return v;
}

// Order-preserving float <-> uint encoding (for atomic min/max of floats).
__device__ __host__ inline uint32_t f2ord(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __host__ inline float ord2f(uint32_t u) {
    u = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
    return __builtin_bit_cast(float, u);
}

}  // namespace gr
