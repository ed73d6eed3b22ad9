// Ray-packet projection kernels: forward (Eq. 12 with the kappa cutoff),
// backward (gradient of a per-ray loss) and the fused forward -> loss ->
// backward pass.
//
// One wave64 owns one packet of 64 consecutive rays (one lane per ray):
//  1. the rays' bounding "beam" is built once per packet: a frame (a, e1, e2)
//     from the first ray's direction, and per-ray intercepts X and slopes S of
//     every line x(z) = X + z S in that frame, reduced to [min, max] ranges
//     with DPP;
//  2. the wave walks the binary LBVH with a wave-uniform stack kept in one
//     VGPR (a lane per stack slot); node boxes come in with one scalar load
//     and are slab-tested per ray, ballots decide where the wave goes;
//  3. at a leaf, up to 64 Gaussians are tested lane-parallel against the beam
//     (support widths of each kappa ellipsoid along a, e1, e2), giving a
//     64-bit candidate mask;
//  4. for each candidate the 64-byte Gaussian record is fetched with one
//     scalar load and every lane evaluates the closed form for its ray.
//
// Closed form (Sec. 3.2-3.3, Eq. 7-11). With delta = o - mu, the literal
// A = d^T P d, B = d^T P delta, C = delta^T P delta and D = C - B^2/A are
// evaluated in FP64, which runs at the full non-packed FP32 rate on CDNA4:
// delta is exact (FP32 inputs), and the cancellation of C A against B^2 costs
// ~eps64 C/D relative, harmless even for origins hundreds of mm away. Only the
// transcendentals run in FP32: r = rsqrt(A), D = (C A - B^2) r^2,
// T = rho sqrt(2 pi) r exp2(-D log2(e)/2) when D <= kappa^2; the per-ray sum
// accumulates in FP64. A = P : (d d^T) uses per-ray products of d.
//
// Gradient (not in the paper; derived from Eq. 11): with t* = -B/A and
// p = delta + t* d (the line's closest point to mu in the metric P),
//   dT/drho = T/rho, dT/dmu = T P p, dT/dP = -(T/2)(p p^T + d d^T/A)
// (the last by the envelope theorem on D = min_t). The backward is
// Gaussian-major: a packet's candidate Gaussians are collected in LDS, 64 at a
// time one per lane, and each lane loops over the packet's rays (staged in
// LDS, rays with zero weight dropped), summing in registers
//   g_rho = sum w T/rho, m = sum w T p, M = sum w T (p p^T + d d^T / A)
// (10 floats), which it adds to its Gaussian's accumulators with one set of
// float atomics. k_epilogue maps them to mean, scale and quaternion gradients.
#include <float.h>
#include <math.h>

#include <type_traits>

#include "gr_launch.h"

namespace gr {

constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2
constexpr float kSqrt2Pi = 2.5066282746310002f;
constexpr float kBeamAbs = 1e-2f;   // absolute margin of the beam test (mm)
constexpr float kBeamRel = 1e-4f;   // relative margin on support widths and slopes
constexpr float kCosDegenerate = 0.5f;

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------

template <int CTRL, int ROW_MASK = 0xF>
__device__ inline float dpp(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                  __builtin_bit_cast(int, v), CTRL,
                                                                  ROW_MASK, 0xF, false));
}

__device__ inline float lane63(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Sum over the 64 lanes: quad butterflies, row rotations, then row broadcasts
// 15 and 31 carry the row sums into lane 63. All lanes must be active.
__device__ inline float wave_sum(float v) {
    v += dpp<0xB1>(0.0f, v);         // quad_perm [1,0,3,2]
    v += dpp<0x4E>(0.0f, v);         // quad_perm [2,3,0,1]
    v += dpp<0x124>(0.0f, v);        // row_ror:4
    v += dpp<0x128>(0.0f, v);        // row_ror:8
    v += dpp<0x142, 0xA>(0.0f, v);   // row_bcast:15 into rows 1, 3
    v += dpp<0x143, 0xC>(0.0f, v);   // row_bcast:31 into rows 2, 3
    return lane63(v);
}

__device__ inline float wave_min(float v) {
    const float I = INFINITY;
    v = fminf(v, dpp<0xB1>(I, v));
    v = fminf(v, dpp<0x4E>(I, v));
    v = fminf(v, dpp<0x124>(I, v));
    v = fminf(v, dpp<0x128>(I, v));
    v = fminf(v, dpp<0x142, 0xA>(I, v));
    v = fminf(v, dpp<0x143, 0xC>(I, v));
    return lane63(v);
}

__device__ inline float wave_max(float v) { return -wave_min(-v); }

__device__ inline float lane_value(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

__device__ inline float bcast0(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

// Read-only data at a wave-uniform address, through the constant address
// space so that the compiler emits scalar loads into SGPRs.
template <class T>
using const_ptr = const __attribute__((address_space(4))) T *;
template <class T>
__device__ inline T sload(const T *p, int64_t i) {
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const_ptr<T>)p)[i];
#else
    return p[i];  // host pass only parses device code
#endif
}

// ---------------------------------------------------------------------------
// per-lane ray and per-wave beam
// ---------------------------------------------------------------------------

struct Ray {
    float o[3], d[3];
    float inv[3], oinv[3];  // reciprocal direction and o * inv for the slab test
    double o64[3], d64[3];
    double dd[6];           // d d^T products: xx yy zz 2xy 2xz 2yz
};

struct Beam {
    float O[3];
    float a[3], e1[3], e2[3];
    float qa[6], q1[6], q2[6];  // products for the quadratic forms x^T M x
    float X1lo, X1hi, X2lo, X2hi, S1lo, S1hi, S2lo, S2hi;
    bool degenerate;
};

// d d^T products in the order the pair evaluation uses: xx yy zz 2xy 2xz 2yz.
__device__ inline void ray_dd(const double d[3], double dd[6]) {
    dd[0] = d[0] * d[0];
    dd[1] = d[1] * d[1];
    dd[2] = d[2] * d[2];
    dd[3] = 2.0 * d[0] * d[1];
    dd[4] = 2.0 * d[0] * d[2];
    dd[5] = 2.0 * d[1] * d[2];
}

__device__ inline void load_ray(const float *__restrict__ ro, const float *__restrict__ rd,
                                int64_t nr_total, int64_t idx, Ray &R) {
    for (int k = 0; k < 3; ++k) {
        R.o[k] = ro[k * nr_total + idx];
        R.d[k] = rd[k * nr_total + idx];
    }
    for (int k = 0; k < 3; ++k) {
        R.o64[k] = R.o[k];
        R.d64[k] = R.d[k];
        const float iv = R.d[k] != 0.0f ? 1.0f / R.d[k] : copysignf(1e30f, R.d[k]);
        R.inv[k] = iv;
        R.oinv[k] = R.o[k] * iv;
    }
    ray_dd(R.d64, R.dd);
}

__device__ inline void sym_products(const float e[3], float q[6]) {
    q[0] = e[0] * e[0];
    q[1] = e[1] * e[1];
    q[2] = e[2] * e[2];
    q[3] = 2.0f * e[0] * e[1];
    q[4] = 2.0f * e[0] * e[2];
    q[5] = 2.0f * e[1] * e[2];
}

__device__ inline void build_beam(const Ray &R, Beam &B) {
    for (int k = 0; k < 3; ++k) B.O[k] = bcast0(R.o[k]);
    float a[3] = {bcast0(R.d[0]), bcast0(R.d[1]), bcast0(R.d[2])};
    const float an = rsqrtf(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int k = 0; k < 3; ++k) a[k] *= an;
    // e1 perpendicular to a, built from the axis least aligned with a
    const float ax = fabsf(a[0]), ay = fabsf(a[1]), az = fabsf(a[2]);
    float h[3] = {0.0f, 0.0f, 0.0f};
    if (ax <= ay && ax <= az) h[0] = 1.0f; else if (ay <= az) h[1] = 1.0f; else h[2] = 1.0f;
    float e1[3] = {a[1] * h[2] - a[2] * h[1], a[2] * h[0] - a[0] * h[2], a[0] * h[1] - a[1] * h[0]};
    const float e1n = rsqrtf(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int k = 0; k < 3; ++k) e1[k] *= e1n;
    float e2[3] = {a[1] * e1[2] - a[2] * e1[1], a[2] * e1[0] - a[0] * e1[2], a[0] * e1[1] - a[1] * e1[0]};
    for (int k = 0; k < 3; ++k) {
        B.a[k] = a[k];
        B.e1[k] = e1[k];
        B.e2[k] = e2[k];
    }
    sym_products(B.a, B.qa);
    sym_products(B.e1, B.q1);
    sym_products(B.e2, B.q2);
    // the line o + t d as x(z) = X + z S in the frame
    const float c = R.d[0] * a[0] + R.d[1] * a[1] + R.d[2] * a[2];
    const float dn = sqrtf(R.d[0] * R.d[0] + R.d[1] * R.d[1] + R.d[2] * R.d[2]);
    const bool bad = !(fabsf(c) >= kCosDegenerate * dn);
    const float ic = bad ? 0.0f : 1.0f / c;
    const float S1 = (R.d[0] * e1[0] + R.d[1] * e1[1] + R.d[2] * e1[2]) * ic;
    const float S2 = (R.d[0] * e2[0] + R.d[1] * e2[1] + R.d[2] * e2[2]) * ic;
    const float rel[3] = {R.o[0] - B.O[0], R.o[1] - B.O[1], R.o[2] - B.O[2]};
    const float z = rel[0] * a[0] + rel[1] * a[1] + rel[2] * a[2];
    float X1 = rel[0] * e1[0] + rel[1] * e1[1] + rel[2] * e1[2] - z * S1;
    float X2 = rel[0] * e2[0] + rel[1] * e2[1] + rel[2] * e2[2] - z * S2;
    float T1 = S1, T2 = S2;
    B.degenerate = ballot(bad) != 0;
    // Turn (e1, e2) about a so that e1 follows the step from the packet's
    // first ray to its second (a row of a detector tile in the generators'
    // order): the tile's cross-section then sits square in the frame and its
    // bounding rectangle, which the candidate test uses, stays tight.
    {
        const float u1 = lane_value(X1, 1) - lane_value(X1, 0);
        const float u2 = lane_value(X2, 1) - lane_value(X2, 0);
        const float un = u1 * u1 + u2 * u2;
        if (un > 1e-12f) {
            const float inv = rsqrtf(un);
            const float c = u1 * inv, sn = u2 * inv;
            const float x1 = X1, x2 = X2, t1 = T1, t2 = T2;
            X1 = c * x1 + sn * x2;
            X2 = c * x2 - sn * x1;
            T1 = c * t1 + sn * t2;
            T2 = c * t2 - sn * t1;
            float f1[3], f2[3];
            for (int k = 0; k < 3; ++k) {
                f1[k] = c * B.e1[k] + sn * B.e2[k];
                f2[k] = c * B.e2[k] - sn * B.e1[k];
            }
            for (int k = 0; k < 3; ++k) {
                B.e1[k] = f1[k];
                B.e2[k] = f2[k];
            }
            sym_products(B.e1, B.q1);
            sym_products(B.e2, B.q2);
        }
    }
    const float x1lo = wave_min(X1), x1hi = wave_max(X1);
    const float x2lo = wave_min(X2), x2hi = wave_max(X2);
    const float s1lo = wave_min(T1), s1hi = wave_max(T1);
    const float s2lo = wave_min(T2), s2hi = wave_max(T2);
    const float xm1 = kBeamAbs + kBeamRel * fmaxf(fabsf(x1lo), fabsf(x1hi));
    const float xm2 = kBeamAbs + kBeamRel * fmaxf(fabsf(x2lo), fabsf(x2hi));
    const float sm1 = 1e-6f + kBeamRel * fmaxf(fabsf(s1lo), fabsf(s1hi));
    const float sm2 = 1e-6f + kBeamRel * fmaxf(fabsf(s2lo), fabsf(s2hi));
    B.X1lo = x1lo - xm1;
    B.X1hi = x1hi + xm1;
    B.X2lo = x2lo - xm2;
    B.X2hi = x2hi + xm2;
    B.S1lo = s1lo - sm1;
    B.S1hi = s1hi + sm1;
    B.S2lo = s2lo - sm2;
    B.S2hi = s2hi + sm2;
    // every field is the same on all lanes: keep them in scalar registers,
    // which frees ~38 vector registers through the traversal and pair loops
    for (int k = 0; k < 3; ++k) {
        B.O[k] = bcast0(B.O[k]);
        B.a[k] = bcast0(B.a[k]);
        B.e1[k] = bcast0(B.e1[k]);
        B.e2[k] = bcast0(B.e2[k]);
    }
    for (int k = 0; k < 6; ++k) {
        B.qa[k] = bcast0(B.qa[k]);
        B.q1[k] = bcast0(B.q1[k]);
        B.q2[k] = bcast0(B.q2[k]);
    }
    B.X1lo = bcast0(B.X1lo);
    B.X1hi = bcast0(B.X1hi);
    B.X2lo = bcast0(B.X2lo);
    B.X2hi = bcast0(B.X2hi);
    B.S1lo = bcast0(B.S1lo);
    B.S1hi = bcast0(B.S1hi);
    B.S2lo = bcast0(B.S2lo);
    B.S2hi = bcast0(B.S2hi);
}

// Conservative test: can any line of the beam meet the ellipsoid with centre
// c and shape M = kappa^2 Sigma? The ellipsoid spans depths z +- ha; over that
// depth range the beam's transverse coordinates lie in X + z S intervals,
// which must overlap the ellipsoid's transverse extents x +- h.
__device__ inline bool beam_hits(const Beam &B, const float c[3], const float M[6]) {
    const float r[3] = {c[0] - B.O[0], c[1] - B.O[1], c[2] - B.O[2]};
    const float z = r[0] * B.a[0] + r[1] * B.a[1] + r[2] * B.a[2];
    const float x1 = r[0] * B.e1[0] + r[1] * B.e1[1] + r[2] * B.e1[2];
    const float x2 = r[0] * B.e2[0] + r[1] * B.e2[1] + r[2] * B.e2[2];
    auto quad = [&](const float *qq) {
        return M[0] * qq[0] + M[1] * qq[1] + M[2] * qq[2] + M[3] * qq[3] + M[4] * qq[4] + M[5] * qq[5];
    };
    // the hardware square root (about 1 ulp) is well inside the kBeamRel margin
    const float ha = __builtin_amdgcn_sqrtf(fmaxf(quad(B.qa), 0.0f)) * (1.0f + kBeamRel) + kBeamAbs;
    const float h1 = __builtin_amdgcn_sqrtf(fmaxf(quad(B.q1), 0.0f)) * (1.0f + kBeamRel) + kBeamAbs;
    const float h2 = __builtin_amdgcn_sqrtf(fmaxf(quad(B.q2), 0.0f)) * (1.0f + kBeamRel) + kBeamAbs;
    const float zl = z - ha, zh = z + ha;
    const float p1 = zl * B.S1lo, p2 = zl * B.S1hi, p3 = zh * B.S1lo, p4 = zh * B.S1hi;
    const float lo1 = B.X1lo + fminf(fminf(p1, p2), fminf(p3, p4));
    const float hi1 = B.X1hi + fmaxf(fmaxf(p1, p2), fmaxf(p3, p4));
    const float r1 = zl * B.S2lo, r2 = zl * B.S2hi, r3 = zh * B.S2lo, r4 = zh * B.S2hi;
    const float lo2 = B.X2lo + fminf(fminf(r1, r2), fminf(r3, r4));
    const float hi2 = B.X2hi + fmaxf(fmaxf(r1, r2), fmaxf(r3, r4));
    return (x1 + h1 >= lo1) && (x1 - h1 <= hi1) && (x2 + h2 >= lo2) && (x2 - h2 <= hi2);
}

// Slab test of an infinite line against a box (min xyz, max xyz). An empty
// box (min > max) never hits.
__device__ inline bool slab(const float *b, const Ray &R) {
    const float tx0 = fmaf(b[0], R.inv[0], -R.oinv[0]), tx1 = fmaf(b[3], R.inv[0], -R.oinv[0]);
    const float ty0 = fmaf(b[1], R.inv[1], -R.oinv[1]), ty1 = fmaf(b[4], R.inv[1], -R.oinv[1]);
    const float tz0 = fmaf(b[2], R.inv[2], -R.oinv[2]), tz1 = fmaf(b[5], R.inv[2], -R.oinv[2]);
    const float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fminf(tz0, tz1));
    const float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
    return tmin <= tmax && b[0] <= b[3];
}

// ---------------------------------------------------------------------------
// the closed form for one (ray, Gaussian) pair
// ---------------------------------------------------------------------------

// Core of Eq. 7 for one pair, in FP64: delta, P delta, B, C, A and the
// numerator N = C A - B^2 of D = N / A.
struct PairCore {
    double dl[3];  // delta = o - mu
    double B, A, N;
};

__device__ inline void pair_core(const double mu[3], const double P[6], const double o[3],
                                 const double d[3], const double dd[6], PairCore &c) {
    c.dl[0] = o[0] - mu[0];
    c.dl[1] = o[1] - mu[1];
    c.dl[2] = o[2] - mu[2];
    const double px = fma(P[4], c.dl[2], fma(P[3], c.dl[1], P[0] * c.dl[0]));
    const double py = fma(P[5], c.dl[2], fma(P[1], c.dl[1], P[3] * c.dl[0]));
    const double pz = fma(P[2], c.dl[2], fma(P[5], c.dl[1], P[4] * c.dl[0]));
    c.B = fma(d[2], pz, fma(d[1], py, d[0] * px));
    const double C = fma(c.dl[2], pz, fma(c.dl[1], py, c.dl[0] * px));
    c.A = fma(P[5], dd[5], fma(P[4], dd[4], fma(P[3], dd[3], fma(P[2], dd[2], fma(P[1], dd[1], P[0] * dd[0])))));
    c.N = fma(C, c.A, -(c.B * c.B));
}

// D = N / A and r = 1/sqrt(A) in FP32 (one transcendental serves both).
__device__ inline void pair_D(const PairCore &c, float &D, float &r) {
    r = __builtin_amdgcn_rsqf(float(c.A));
    D = (float(c.N) * r) * r;
}

__device__ inline float gauss_exp(float D) { return __builtin_amdgcn_exp2f(-kHalfLog2e * D); }

// ---------------------------------------------------------------------------
// traversal
// ---------------------------------------------------------------------------

// Candidates of leaf l for this packet, as a 64-bit mask over its Gaussians.
__device__ inline uint64_t leaf_candidates(const SceneView &S, const Beam &B, int l, int lane,
                                           int64_t &start) {
    start = int64_t(l) * S.leaf;
    const int64_t rem = S.n - start;
    const int cnt = rem < S.leaf ? int(rem) : S.leaf;
    bool cand = false;
    if (lane < cnt) {
        const int64_t g = start + lane;
        const float c[3] = {S.cull[g], S.cull[S.n + g], S.cull[2 * S.n + g]};
        const float M[6] = {S.cull[3 * S.n + g], S.cull[4 * S.n + g], S.cull[5 * S.n + g],
                            S.cull[6 * S.n + g], S.cull[7 * S.n + g], S.cull[8 * S.n + g]};
        cand = B.degenerate ? true : beam_hits(B, c, M);
    }
    return ballot(cand);
}

template <class LeafFn>
__device__ inline void traverse(const SceneView &S, const Ray &R, bool active, int lane,
                                LeafFn &&leaf_fn) {
    const AccelHeader *hdr = S.hdr;
    const AccelHeader H = sload(hdr, 0);
    const int root = H.root;
    float rb[6];
    for (int k = 0; k < 6; ++k) rb[k] = H.root_box[k];
    if (ballot(active && slab(rb, R)) == 0) return;
    if (root < 0) {
        if (~root < S.n_leaves) leaf_fn(~root);
        return;
    }
    int stack = 0;  // lane k holds stack slot k
    int sp = 0;
    int node = root;
    int32_t err = 0;
    // every node is entered at most once per packet, so this cap is never
    // reached on a well-formed tree; it bounds the loop if the tree is corrupt
    const int64_t cap = 2 * int64_t(S.n_nodes) + 2;
    for (int64_t it = 0;; ++it) {
        if (it >= cap || node < 0 || node >= S.n_nodes) {
            err |= it >= cap ? kFlagTraversalCap : kFlagTreeCorrupt;
            break;
        }
        const Node nd = sload(S.nodes, node);
        const bool h0 = active && slab(nd.b, R);
        const bool h1 = active && slab(nd.b + 6, R);
        const uint64_t m0 = ballot(h0), m1 = ballot(h1);
        const int c0 = nd.child[0];
        const int c1 = nd.child[1];
        int next = -1;
        bool have = false;
        int lv0 = -1, lv1 = -1;  // leaves to visit from this node
        if (m0) {
            if (c0 < 0) {
                if (~c0 < S.n_leaves) lv0 = ~c0; else err |= kFlagTreeCorrupt;
            } else {
                next = c0;
                have = true;
            }
        }
        if (m1) {
            if (c1 < 0) {
                if (~c1 < S.n_leaves) lv1 = ~c1; else err |= kFlagTreeCorrupt;
            } else if (!have) {
                next = c1;
                have = true;
            } else if (sp < 64) {
                stack = (lane == sp) ? c1 : stack;
                ++sp;
            } else {
                err |= kFlagStackOverflow;
            }
        }
        for (int k = 0; k < 2; ++k) {
            const int lf = k == 0 ? lv0 : lv1;
            if (lf >= 0) leaf_fn(lf);
        }
        if (!have) {
            if (sp == 0) break;
            --sp;
            next = __builtin_amdgcn_readlane(stack, sp);
        }
        node = next;
    }
    if (err && lane == 0) atomicOr(const_cast<int32_t *>(&hdr->flags), err);
}

// Conservative beam test of an axis-aligned box (lo, hi): the box's extents
// along a, e1, e2 are the dot products of its half extents with |a|, |e1|, |e2|.
__device__ inline bool beam_box(const Beam &B, const float lo[3], const float hi[3]) {
    if (!(lo[0] <= hi[0])) return false;  // empty box
    if (B.degenerate) return true;
    float c[3], h[3];
    for (int k = 0; k < 3; ++k) {
        c[k] = 0.5f * (lo[k] + hi[k]) - B.O[k];
        h[k] = 0.5f * (hi[k] - lo[k]);
    }
    const float z = c[0] * B.a[0] + c[1] * B.a[1] + c[2] * B.a[2];
    const float x1 = c[0] * B.e1[0] + c[1] * B.e1[1] + c[2] * B.e1[2];
    const float x2 = c[0] * B.e2[0] + c[1] * B.e2[1] + c[2] * B.e2[2];
    const float ha = (h[0] * fabsf(B.a[0]) + h[1] * fabsf(B.a[1]) + h[2] * fabsf(B.a[2])) * (1.0f + kBeamRel) + kBeamAbs;
    const float h1 = (h[0] * fabsf(B.e1[0]) + h[1] * fabsf(B.e1[1]) + h[2] * fabsf(B.e1[2])) * (1.0f + kBeamRel) + kBeamAbs;
    const float h2 = (h[0] * fabsf(B.e2[0]) + h[1] * fabsf(B.e2[1]) + h[2] * fabsf(B.e2[2])) * (1.0f + kBeamRel) + kBeamAbs;
    const float zl = z - ha, zh = z + ha;
    const float p1 = zl * B.S1lo, p2 = zl * B.S1hi, p3 = zh * B.S1lo, p4 = zh * B.S1hi;
    const float lo1 = B.X1lo + fminf(fminf(p1, p2), fminf(p3, p4));
    const float hi1 = B.X1hi + fmaxf(fmaxf(p1, p2), fmaxf(p3, p4));
    const float r1 = zl * B.S2lo, r2 = zl * B.S2hi, r3 = zh * B.S2lo, r4 = zh * B.S2hi;
    const float lo2 = B.X2lo + fminf(fminf(r1, r2), fminf(r3, r4));
    const float hi2 = B.X2hi + fmaxf(fmaxf(r1, r2), fmaxf(r3, r4));
    return (x1 + h1 >= lo1) && (x1 - h1 <= hi1) && (x2 + h2 >= lo2) && (x2 - h2 <= hi2);
}

// Node count and offset of level lv of the wide hierarchy (level 0 = leaves;
// each level above has ceil(count / 64) nodes), from wave-uniform scalars.
__device__ inline void level_info(int n_leaves, int lv, int &cnt, int &off) {
    cnt = n_leaves;
    off = 0;
    for (int k = 0; k < lv; ++k) {
        off += cnt;
        cnt = (cnt + kWide - 1) / kWide;
    }
}

// Ballot over up to 64 consecutive nodes [first, first + cnt) of one level of
// the wide hierarchy: lane k tests node first + k against the beam.
__device__ inline uint64_t wide_children(const SceneView &S, const Beam &B, int level_off, int first,
                                         int cnt, int lane) {
    bool hit = false;
    if (lane < cnt) {
        const int64_t i = int64_t(level_off) + first + lane;
        const int64_t t = S.wide_total;
        const float lo[3] = {S.wbox[i], S.wbox[t + i], S.wbox[2 * t + i]};
        const float hi[3] = {S.wbox[3 * t + i], S.wbox[4 * t + i], S.wbox[5 * t + i]};
        hit = beam_box(B, lo, hi);
    }
    return ballot(hit);
}

// per-wave LDS stack entries: a popped node pushes at most 64 children, so the
// depth never exceeds 64 per level below the top
constexpr int kWideStack = 64 * (kMaxLevels - 1);

// Packet traversal of the wide hierarchy with beam tests, 64 boxes per wave
// step. Pending internal nodes wait on a per-wave LDS stack (entry = level in
// the top 4 bits, node index below); leaves are handed to leaf_fn as soon as
// their parent's ballot names them, from a single call site.
template <class LeafFn>
__device__ inline void traverse_wide(const SceneView &S, const Beam &B, bool any_active, int lane,
                                     uint32_t *stack, LeafFn &&leaf_fn) {
    if (!any_active) return;
    const int top = S.n_levels - 1;
    int n_top, top_off;
    level_info(S.n_leaves, top, n_top, top_off);
    int sp = 0;          // wave-uniform stack depth
    int next_root = 0;   // next chunk of top-level nodes (children of a virtual root)
    int32_t err = 0;
    while (true) {
        int lv, first, cnt, off;
        if (sp > 0) {
            --sp;
            const uint32_t e = uint32_t(__builtin_amdgcn_readfirstlane(int(stack[sp])));
            lv = int(e >> 28) - 1;  // children of a node at level (e >> 28)
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
        uint64_t mask = wide_children(S, B, off, first, cnt, lane);
        if (lv == 0) {
            while (mask) {
                const int c = first + __builtin_ctzll(mask);
                mask &= mask - 1;
                leaf_fn(c);
            }
        } else {
            const int nh = __builtin_popcountll(mask);
            if (sp + nh > kWideStack) {
                err |= kFlagStackOverflow;
                continue;
            }
            // lowest child on top of the stack, so children are visited in order
            if ((mask >> lane) & 1ull) {
                const int above = __builtin_popcountll(mask >> lane) - 1;
                stack[sp + above] = (uint32_t(lv) << 28) | uint32_t(first + lane);
            }
            __builtin_amdgcn_wave_barrier();
            sp += nh;
        }
    }
    if (err && lane == 0) atomicOr(const_cast<int32_t *>(&S.hdr->flags), err);
}

// Traversal dispatch: 2 = wide hierarchy (default), 1 = binary LBVH.
template <class LeafFn>
__device__ inline void traverse_any(int mode, const SceneView &S, const Ray &R, const Beam &B,
                                    bool active, int lane, uint32_t *stack, LeafFn &&leaf_fn) {
    if (mode == 1)
        traverse(S, R, active, lane, leaf_fn);
    else
        traverse_wide(S, B, ballot(active) != 0, lane, stack, leaf_fn);
}

__device__ inline int64_t logical_block(int xcd_remap) {
    const int64_t b = blockIdx.x;
    if (xcd_remap == 2) return b;
    const int64_t G = gridDim.x, nx = 8;
    const int64_t per = G / nx, rem = G % nx;
    const int64_t x = b % nx, k = b / nx;
    return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// Locates this wave's packet: its segment, and the lane's ray and output.
struct PacketRef {
    int seg;
    int64_t ray;   // index of this lane's ray in the segment's arrays (the packet's first
                   // ray when the lane is past the segment's end)
    int64_t out;   // output index of this lane
    bool active;
};

__device__ inline bool locate_packet(const LaunchTable &T, int64_t packet, int lane, PacketRef &P) {
    if (packet >= T.n_packets) return false;
    int s = 0;
    for (int k = 1; k < T.n_segs; ++k)
        if (packet >= T.segs[k].first_packet) s = k;
    const Segment &sg = T.segs[s];
    const int64_t local0 = (packet - sg.first_packet) * 64;
    const int64_t local = local0 + lane;
    P.seg = s;
    P.active = local < sg.n_rays;
    P.ray = sg.ray_offset + (P.active ? local : local0);
    P.out = sg.out_offset + local;
    return true;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Forward sum over one leaf's candidate Gaussians (mask), two records per
// step: both scalar loads are in flight before the first evaluation, so one
// load latency is exposed per two pairs.
template <bool kStats>
__device__ inline void leaf_forward(const SceneView &S, const Ray &R, int64_t start, uint64_t mask,
                                    float k2, bool active, double &acc, uint32_t &n_inc,
                                    uint32_t &n_hitc) {
    while (mask) {
        const int j0 = __builtin_ctzll(mask);
        mask &= mask - 1;
        const bool two = mask != 0;
        const int j1 = two ? __builtin_ctzll(mask) : j0;
        if (two) mask &= mask - 1;
        const GaussRec G0 = sload(S.rec, start + j0);
        const GaussRec G1 = sload(S.rec, start + j1);
        PairCore c;
        float D, r;
        pair_core(G0.mu, G0.P, R.o64, R.d64, R.dd, c);
        pair_D(c, D, r);
        if (kStats) n_hitc += ballot(active && D <= k2) != 0 ? 1u : 0u;
        if (D <= k2) {
            acc += double(G0.rho_c * r * gauss_exp(D));
            if (kStats) n_inc += active ? 1u : 0u;
        }
        if (two) {
            pair_core(G1.mu, G1.P, R.o64, R.d64, R.dd, c);
            pair_D(c, D, r);
            if (kStats) n_hitc += ballot(active && D <= k2) != 0 ? 1u : 0u;
            if (D <= k2) {
                acc += double(G1.rho_c * r * gauss_exp(D));
                if (kStats) n_inc += active ? 1u : 0u;
            }
        }
    }
}

// One packet of the forward pass. kStats adds work counters (atomics once per
// packet) for measurement runs; the production instantiation has none.
template <bool kStats>
__device__ inline void packet_forward(const LaunchTable &T, int64_t packet, int lane, uint32_t *stack,
                                      uint64_t *stats) {
    PacketRef P;
    if (!locate_packet(T, packet, lane, P)) return;
    const Segment &sg = T.segs[P.seg];
    const SceneView S = T.scenes[sg.scene];
    float *out = sg.out;
    Ray R;
    load_ray(sg.ro, sg.rd, sg.stride, P.ray, R);
    Beam B;
    build_beam(R, B);
    double acc = 0.0;
    const float k2 = S.kappa2;
    uint32_t n_inc = 0, n_cand = 0, n_leaf = 0, n_hitc = 0;
    traverse_any(T.traversal, S, R, B, P.active, lane, stack, [&](int l) {
        int64_t start;
        const uint64_t mask = leaf_candidates(S, B, l, lane, start);
        if (kStats) {
            ++n_leaf;
            n_cand += __builtin_popcountll(mask);
        }
        leaf_forward<kStats>(S, R, start, mask, k2, P.active, acc, n_inc, n_hitc);
    });
    if (P.active) out[P.out] = float(acc);
    if (kStats) {
        const float inc = wave_sum(float(n_inc));
        const uint64_t act = ballot(P.active);
        if (lane == 0) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&stats[0]), (unsigned long long)(inc));
            atomicAdd(reinterpret_cast<unsigned long long *>(&stats[1]),
                      (unsigned long long)(n_cand) * (unsigned long long)(__builtin_popcountll(act)));
            atomicAdd(reinterpret_cast<unsigned long long *>(&stats[2]), (unsigned long long)(n_leaf));
            atomicAdd(reinterpret_cast<unsigned long long *>(&stats[3]), 1ull);
            atomicAdd(reinterpret_cast<unsigned long long *>(&stats[4]), (unsigned long long)(n_cand));
            atomicAdd(reinterpret_cast<unsigned long long *>(&stats[5]), (unsigned long long)(n_hitc));
        }
    }
}

// Next packet of a persistent launch: lane 0 takes a ticket from the work
// counter and the wave shares it.
__device__ inline int64_t next_packet(uint32_t *counter, int lane) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(counter, 1u);
    return int64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(t))));
}

template <bool kStats>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5))) void k_forward(
    LaunchTable T, uint64_t *stats) {
    extern __shared__ uint32_t fwd_stack[];  // kWideStack entries per wave
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    uint32_t *stack = fwd_stack + wave * kWideStack;
    if (T.work_counter) {
        // persistent: waves pull packets until the table is exhausted
        for (int64_t packet = next_packet(T.work_counter, lane); packet < T.n_packets;
             packet = next_packet(T.work_counter, lane))
            packet_forward<kStats>(T, packet, lane, stack, stats);
        return;
    }
    const int64_t packet = logical_block(T.xcd_remap) * T.waves_per_group + wave;
    packet_forward<kStats>(T, packet, lane, stack, stats);
}

// Per-ray record staged in LDS for the backward (56 bytes: a stride of 14
// dwords spreads the rays of a packet over the LDS banks when lanes gather
// different rays). d d^T is recomputed from d where needed.
struct RayRec {
    double o[3];
    double d[3];
    float w;        // dL/dI of the ray
    float pad;
};
static_assert(sizeof(RayRec) == 56, "RayRec must be 56 bytes");

// A ray as its lane holds it for the backward: the FP32 inputs (exact in
// FP64) and the weight dL/dI.
struct RayF {
    float o[3], d[3];
    float w;
};

__device__ inline RayRec widen(const RayF &f) {
    RayRec r;
    for (int k = 0; k < 3; ++k) {
        r.o[k] = double(f.o[k]);
        r.d[k] = double(f.d[k]);
    }
    r.w = f.w;
    r.pad = 0.0f;
    return r;
}

// Ray i from the lane that holds it (ds_bpermute; every lane of the wave must
// execute this). i is per lane.
__device__ inline RayRec gather_ray(const RayF &mine, int i) {
    const int a = i << 2;
    auto g = [&](float v) {
        return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(a, __builtin_bit_cast(int, v)));
    };
    RayF f;
    for (int k = 0; k < 3; ++k) {
        f.o[k] = g(mine.o[k]);
        f.d[k] = g(mine.d[k]);
    }
    f.w = g(mine.w);
    return widen(f);
}

// Ray i, the same on every lane (v_readlane into scalars).
__device__ inline RayRec lane_ray(const RayF &mine, int i) {
    auto r = [&](float v) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), i));
    };
    RayF f;
    for (int k = 0; k < 3; ++k) {
        f.o[k] = r(mine.o[k]);
        f.d[k] = r(mine.d[k]);
    }
    f.w = r(mine.w);
    return widen(f);
}

constexpr int kCandCap = 128;  // candidate list slots per wave (a batch is 64)

// One window of up to kWin hit-list entries being replayed (non-empty ones
// only, in list order): records, masks, Gaussian indices, inclusive prefix
// sums of the pair counts, and the per-entry gradient sums (SoA,
// res[k][entry]). 48 entries keep the per-wave LDS at 10 KB, so that the
// fused kernel's occupancy stays bounded by registers, not LDS.
constexpr int kWin = 64;
constexpr int kWinLog2 = 6;  // search steps: 2^6 >= kWin
struct HitWindow {
    GaussRec rec[kWin];
    float res[10][kWin];
    uint64_t m[kWin];
    int32_t g[kWin];
    int32_t incl[kWin];
};

// Traversal stack and candidate list of the re-traversal backward.
struct TravLds {
    int32_t cand[kCandCap];
    uint32_t stack[kWideStack];
};

// Per-wave LDS of the fused kernel: the rays stay in their lanes (gathered
// with bpermute / readlane), so the whole budget goes to the replay window.
struct WaveLdsFused {
    union {
        TravLds t;      // traversal and re-traversal backward
        HitWindow win;  // hit-list replay (the traversal is over by then)
    };
};

// Per-wave LDS of the backward with dL/dI given: the weighted rays staged at
// their lane's slot, read by all lanes at once in the Gaussian-major batches.
struct WaveLdsPlain {
    RayRec rays[64];
    TravLds t;
};

// Where a batch reads ray i from (i is the same on every lane).
struct RaysInLds {
    const RayRec *rays;
    __device__ RayRec get(int i) const { return rays[i]; }
};
struct RaysInLanes {
    const RayF &mine;
    __device__ RayRec get(int i) const { return lane_ray(mine, i); }
};

// Gradient terms of one (ray, Gaussian) pair added to the ten accumulators
// c = (sum w E, sum wT p, sum of the symmetric wT (p p^T + d d^T / A)) that the
// epilogue turns into parameter gradients; E is the unit-density integral
// sqrt(2 pi / A) exp(-D/2) and T = rho E. Returns whether the pair is inside
// the cutoff (D <= kappa^2).
__device__ inline bool pair_grad(const double mu[3], const double P[6], float rho, const RayRec &Rr, float k2,
                                 float c[10]) {
    double dd[6];
    ray_dd(Rr.d, dd);
    PairCore pc;
    pair_core(mu, P, Rr.o, Rr.d, dd, pc);
    float D, r;
    pair_D(pc, D, r);
    if (!(D <= k2)) return false;
    // p = delta - (B/A) d in FP64 (t = B/A can be hundreds of mm);
    // 1/A from the FP32 r^2 (relative error ~1e-7) and one Newton step
    double ra = double(r * r);
    ra = fma(ra, fma(-pc.A, ra, 1.0), ra);
    const double t = pc.B * ra;
    const float p0 = float(fma(-t, Rr.d[0], pc.dl[0]));
    const float p1 = float(fma(-t, Rr.d[1], pc.dl[1]));
    const float p2 = float(fma(-t, Rr.d[2], pc.dl[2]));
    const float wE = Rr.w * (kSqrt2Pi * r * gauss_exp(D));
    const float wT = wE * rho;
    const float wTA = wT * (r * r);
    const float q0 = wT * p0, q1 = wT * p1, q2 = wT * p2;
    const float f0 = float(Rr.d[0]), f1 = float(Rr.d[1]), f2 = float(Rr.d[2]);  // exact (FP32 input)
    const float v0 = wTA * f0, v1 = wTA * f1, v2 = wTA * f2;
    c[0] += wE;
    c[1] += q0;
    c[2] += q1;
    c[3] += q2;
    c[4] = fmaf(q0, p0, fmaf(v0, f0, c[4]));
    c[5] = fmaf(q1, p1, fmaf(v1, f1, c[5]));
    c[6] = fmaf(q2, p2, fmaf(v2, f2, c[6]));
    c[7] = fmaf(q0, p1, fmaf(v0, f1, c[7]));
    c[8] = fmaf(q0, p2, fmaf(v0, f2, c[8]));
    c[9] = fmaf(q1, p2, fmaf(v1, f2, c[9]));
    return true;
}

__device__ inline void flush_grad(float *acc, int64_t n, int64_t g, float c[10]) {
    for (int k = 0; k < 10; ++k) {
        atomicAdd(&acc[k * n + g], c[k]);
        c[k] = 0.0f;
    }
}

// One batch of up to 64 candidate Gaussians (lane j owns cand[j]) against the
// packet's staged rays (the set bits of live).
template <class Rays>
__device__ inline void backward_batch(const SceneView &S, const TravLds &Lt, const Rays &rays, int cnt,
                                      uint64_t live, int lane, float k2, float *acc) {
    const bool own = lane < cnt;
    const int64_t g = own ? Lt.cand[lane] : Lt.cand[0];
    const GaussRec G = S.rec[g];
    const float rho = G.rho_c * (1.0f / kSqrt2Pi);
    float c[10];
    for (int k = 0; k < 10; ++k) c[k] = 0.0f;
    bool any = false;
    for (uint64_t lm = live; lm; lm &= lm - 1) {
        const int i = __builtin_ctzll(lm);
        any |= pair_grad(G.mu, G.P, rho, rays.get(i), k2, c);
    }
    if (own && any) flush_grad(acc, S.n, g, c);
}

// Hit list of one packet: (Gaussian, 64-bit mask of the packet's rays with
// D <= kappa^2) for every candidate with at least one such ray, recorded by
// the forward half of the fused pass into this wave's region of the caller's
// scratch (cap entries). Entries collect in registers (lane k holds the k-th
// pending one) and go out 64 at a time as coalesced stores. A packet with
// more than cap entries marks the list overflowed; its backward half then
// falls back to re-traversal.
struct HitList {
    uint32_t *g;
    uint64_t *m;
    int cap;
    int n;        // entries stored (wave-uniform)
    int nbuf;     // entries pending in registers (wave-uniform)
    bool overflow;
    uint32_t bg;  // this lane's pending entry
    uint64_t bm;

    __device__ void flush(int lane) {
        if (nbuf == 0) return;
        if (n + nbuf <= cap) {
            if (lane < nbuf) {
                g[n + lane] = bg;
                m[n + lane] = bm;
            }
            n += nbuf;
        } else {
            overflow = true;
        }
        nbuf = 0;
    }
    // Appends (gi, mask) when mask is non-zero. The append itself is
    // branch-free (selects); only the store of a full batch branches.
    __device__ void record(int lane, int64_t gi, uint64_t mask) {
        const bool put = mask != 0 && !overflow && lane == nbuf;
        bg = put ? uint32_t(gi) : bg;
        bm = put ? mask : bm;
        nbuf += (mask != 0 && !overflow) ? 1 : 0;
        if (nbuf == 64) flush(lane);
    }
};

// Forward sum over one leaf's candidates (as leaf_forward), also recording the
// packet's hit list.
__device__ inline void leaf_forward_hits(const SceneView &S, const Ray &R, int64_t start, uint64_t mask,
                                         float k2, bool active, double &acc, HitList &H, int lane) {
    while (mask) {
        const int j0 = __builtin_ctzll(mask);
        mask &= mask - 1;
        const bool two = mask != 0;
        const int j1 = two ? __builtin_ctzll(mask) : j0;
        if (two) mask &= mask - 1;
        const GaussRec G0 = sload(S.rec, start + j0);
        const GaussRec G1 = sload(S.rec, start + j1);
        PairCore c;
        float D, r;
        pair_core(G0.mu, G0.P, R.o64, R.d64, R.dd, c);
        pair_D(c, D, r);
        const uint64_t h0 = ballot(active && D <= k2);
        if (D <= k2) acc += double(G0.rho_c * r * gauss_exp(D));
        if (h0) H.record(lane, start + j0, h0);
        if (two) {
            pair_core(G1.mu, G1.P, R.o64, R.d64, R.dd, c);
            pair_D(c, D, r);
            const uint64_t h1 = ballot(active && D <= k2);
            if (D <= k2) acc += double(G1.rho_c * r * gauss_exp(D));
            if (h1) H.record(lane, start + j1, h1);
        }
    }
}

// m without its r lowest set bits (0 <= r < popcount(m)): the position of the
// r-th set bit by halving, then a mask.
__device__ inline uint64_t drop_low_bits(uint64_t m, int r) {
    uint64_t x = m;
    int pos = 0;
    for (int w = 32; w >= 1; w >>= 1) {
        const int low = __builtin_popcountll(x & ((1ull << w) - 1ull));
        const bool up = r >= low;
        r = up ? r - low : r;
        x = up ? x >> w : x;
        pos = up ? pos + w : pos;
    }
    return m & (~0ull << pos);
}

// Inclusive prefix sum over the wave (lane k gets the sum of lanes 0..k):
// shifts by 1, 2, 4, 8 within each row of 16 lanes, then the row totals
// (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3).
__device__ inline int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);
    return v;
}

// Backward half from a recorded hit list, in windows of kWin entries. The T
// included pairs of a window are split evenly over the lanes (lane k takes
// pairs [k s, k s + s) of the window's pairs in list order, s = ceil(T / 64)),
// so every lane is busy however unequal the entries' ray counts are. A lane
// adds its partial sums for an entry into the window's LDS sums when it moves
// on; at the end of the window lane j adds entry j's sums to the global
// accumulators, so those atomics cover consecutive Gaussians of the same
// leaves. The next window's entries are loaded while the current window runs.
__device__ inline void drain_hits(const SceneView &S, WaveLdsFused *L, const RayF &mine, const uint32_t *hg,
                                  const uint64_t *hm, int n_ent, uint64_t live, int lane, float k2,
                                  float *acc) {
    const int64_t n = S.n;
    HitWindow &W = L->win;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    // entries (pg, pm) of the next window, in flight
    uint32_t pg = 0;
    uint64_t pm = 0;
    if (lane < min(kWin, n_ent)) {
        pg = hg[lane];
        pm = hm[lane] & live;
    }
    for (int e0 = 0; e0 < n_ent; e0 += kWin) {
        const int64_t gj = pg;
        const uint64_t mj = pm;
        const int e1 = e0 + kWin;
        pm = 0;
        if (lane < min(kWin, n_ent - e1)) {
            pg = hg[e1 + lane];
            pm = hm[e1 + lane] & live;
        }
        const int cj = __builtin_popcountll(mj);
        const int incl = wave_incl_scan(cj);
        const int T = __builtin_amdgcn_readlane(incl, 63);
        if (T == 0) continue;
        // compact the entries with pairs into slots 0..nq-1
        const uint64_t nonempty = ballot(cj > 0);
        const int nq = __builtin_popcountll(nonempty);
        if (cj > 0) {
            const int q = __builtin_popcountll(nonempty & below);
            W.rec[q] = S.rec[gj];
            W.m[q] = mj;
            W.g[q] = int32_t(gj);
            W.incl[q] = incl;
        }
        if (lane < kWin)
            for (int k = 0; k < 10; ++k) W.res[k][lane] = 0.0f;
        __builtin_amdgcn_wave_barrier();
        const int inclq = lane < nq ? W.incl[lane] : T;
        // this lane's pairs: [p, p + left) of the window's T pairs
        const int s = (T + 63) >> 6;
        const int p = lane * s;
        const int left = max(0, min(s, T - p));
        // first slot whose inclusive count exceeds p (binary search over lanes)
        int lo = 0, hi = kWin - 1;
        for (int step = 0; step < kWinLog2; ++step) {
            const int mid = (lo + hi) >> 1;
            const int v = __shfl(inclq, mid, 64);
            if (v > p) hi = mid; else lo = mid + 1;
        }
        int e = left > 0 ? lo : 0;
        uint64_t m = W.m[e];
        // skip the entry's first (p - exclusive prefix) rays
        if (left > 0) m = drop_low_bits(m, p - (W.incl[e] - __builtin_popcountll(m)));
        GaussRec G = W.rec[e];
        float rho = G.rho_c * (1.0f / kSqrt2Pi);
        float c[10];
        for (int k = 0; k < 10; ++k) c[k] = 0.0f;
        for (int it = 0; it < s; ++it) {
            const bool act = it < left;
            if (act && m == 0) {
                // entry done: add its partial sums to the window's, take the next
                for (int k = 0; k < 10; ++k) {
                    atomicAdd(&W.res[k][e], c[k]);
                    c[k] = 0.0f;
                }
                e = min(e + 1, nq - 1);
                m = W.m[e];
                G = W.rec[e];
                rho = G.rho_c * (1.0f / kSqrt2Pi);
            }
            // the gather runs on every lane (bpermute needs its sources active)
            const int i = act ? __builtin_ctzll(m) : lane;
            const RayRec Rr = gather_ray(mine, i);
            if (act) {
                m &= m - 1;
                pair_grad(G.mu, G.P, rho, Rr, k2, c);
            }
        }
        if (left > 0)
            for (int k = 0; k < 10; ++k) atomicAdd(&W.res[k][e], c[k]);
        __builtin_amdgcn_wave_barrier();
        if (lane < nq) {
            const int64_t gq = W.g[lane];
            for (int k = 0; k < 10; ++k) atomicAdd(&acc[k * n + gq], W.res[k][lane]);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Per-ray loss weight dL/dI and loss term for the fused pass.
__device__ inline float loss_weight(int kind, float I, float y, float b, double &term) {
    if (kind == GR_LOSS_L2) {
        const float e = I - y;
        term = 0.5 * double(e) * double(e);
        return e;
    }
    const double Ib = double(I) + double(b);
    term = Ib - double(y) * log(Ib);
    return float(1.0 - double(y) / Ib);
}

// Gaussian-major backward of one packet by re-traversal: the candidates of the
// traversal go into the per-wave LDS list; every 64 of them are one batch.
template <class Rays>
__device__ inline void retraverse_backward(const LaunchTable &T, const SceneView &S, const Ray &R,
                                           const Beam &B, TravLds &Lt, const Rays &rays, uint64_t live_mask,
                                           bool live, int lane, float k2, float *acc) {
    int count = 0;  // wave-uniform number of listed candidates
    traverse_any(T.traversal, S, R, B, live, lane, Lt.stack, [&](int l) {
        int64_t start;
        const uint64_t mask = leaf_candidates(S, B, l, lane, start);
        if (!mask) return;
        if ((mask >> lane) & 1ull) {
            const int pos = count + __builtin_popcountll(mask & ((1ull << lane) - 1ull));
            Lt.cand[pos] = int32_t(start + lane);
        }
        count += __builtin_popcountll(mask);
        __builtin_amdgcn_wave_barrier();
        if (count >= 64) {
            backward_batch(S, Lt, rays, 64, live_mask, lane, k2, acc);
            const int rest = count - 64;
            int moved = 0;
            if (lane < rest) moved = Lt.cand[64 + lane];
            __builtin_amdgcn_wave_barrier();
            if (lane < rest) Lt.cand[lane] = moved;
            __builtin_amdgcn_wave_barrier();
            count = rest;
        }
    });
    if (count > 0) backward_batch(S, Lt, rays, count, live_mask, lane, k2, acc);
}

template <bool kFused>
using WaveLdsOf = typename std::conditional<kFused, WaveLdsFused, WaveLdsPlain>::type;

template <bool kFused>
__device__ inline void packet_backward(const LaunchTable &T, int64_t packet, int lane, WaveLdsOf<kFused> *L,
                                       const BwdArgs &A, uint32_t *hit_g, uint64_t *hit_m) {
    PacketRef P;
    if (!locate_packet(T, packet, lane, P)) return;
    const Segment &sg = T.segs[P.seg];
    const SceneView S = T.scenes[sg.scene];
    Ray R;
    load_ray(sg.ro, sg.rd, sg.stride, P.ray, R);
    Beam B;
    build_beam(R, B);
    const float k2 = S.kappa2;
    float *acc = A.acc;
    if constexpr (kFused) {
        bool listed = false;  // the forward half recorded a complete hit list
        int n_ent = 0;
        double sum = 0.0;
        if (T.hit_cap > 0 && hit_g) {
            HitList H{hit_g, hit_m, T.hit_cap, 0, 0, false, 0u, 0ull};
            traverse_any(T.traversal, S, R, B, P.active, lane, L->t.stack, [&](int l) {
                int64_t start;
                const uint64_t mask = leaf_candidates(S, B, l, lane, start);
                leaf_forward_hits(S, R, start, mask, k2, P.active, sum, H, lane);
            });
            H.flush(lane);
            listed = !H.overflow;
            n_ent = H.n;
        } else {
            uint32_t dummy = 0, dummy2 = 0;
            traverse_any(T.traversal, S, R, B, P.active, lane, L->t.stack, [&](int l) {
                int64_t start;
                const uint64_t mask = leaf_candidates(S, B, l, lane, start);
                leaf_forward<false>(S, R, start, mask, k2, P.active, sum, dummy, dummy2);
            });
        }
        const float I = float(sum);
        double term = 0.0;
        float w = 0.0f;
        if (P.active) {
            w = loss_weight(A.loss_kind, I, A.target[P.out], A.background, term);
            if (A.out_proj) A.out_proj[P.out] = I;
        }
        if (A.out_loss) {
            for (int off = 32; off >= 1; off >>= 1) term += __shfl_xor(term, off);
            if (lane == 0) atomicAdd(A.out_loss, term);
        }
        const bool live = P.active && w != 0.0f;
        const uint64_t live_mask = ballot(live);
        if (live_mask == 0) return;
        // this lane's ray, handed to other lanes by bpermute / readlane
        RayF mine;
        for (int k = 0; k < 3; ++k) {
            mine.o[k] = R.o[k];
            mine.d[k] = R.d[k];
        }
        mine.w = live ? w : 0.0f;
        if (listed) {
            // the list's global stores (other lanes' entries) are visible to
            // this wave's loads after a workgroup-scope release/acquire
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            drain_hits(S, L, mine, hit_g, hit_m, n_ent, live_mask, lane, k2, acc);
            return;
        }
        retraverse_backward(T, S, R, B, L->t, RaysInLanes{mine}, live_mask, live, lane, k2, acc);
    } else {
        const float w = P.active ? A.grad_out[P.out] : 0.0f;
        const bool live = P.active && w != 0.0f;
        const uint64_t live_mask = ballot(live);
        if (live_mask == 0) return;
        // stage the weighted rays, each at its lane's slot
        if (live) {
            RayRec &rr = L->rays[lane];
            for (int k = 0; k < 3; ++k) {
                rr.o[k] = R.o64[k];
                rr.d[k] = R.d64[k];
            }
            rr.w = w;
        }
        __builtin_amdgcn_wave_barrier();
        retraverse_backward(T, S, R, B, L->t, RaysInLds{L->rays}, live_mask, live, lane, k2, acc);
    }
}

template <bool kFused>
__global__ __launch_bounds__(1024) void k_backward(LaunchTable T, BwdArgs A) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    WaveLdsOf<kFused> *L = reinterpret_cast<WaveLdsOf<kFused> *>(lds_raw) + wave;
    if (T.work_counter) {
        // hit-list regions belong to persistent waves (one per wave slot)
        const int64_t slot = int64_t(blockIdx.x) * T.waves_per_group + wave;
        uint32_t *hg = T.hit_cap > 0 ? T.hit_g + slot * T.hit_cap : nullptr;
        uint64_t *hm = T.hit_cap > 0 ? T.hit_m + slot * T.hit_cap : nullptr;
        for (int64_t packet = next_packet(T.work_counter, lane); packet < T.n_packets;
             packet = next_packet(T.work_counter, lane))
            packet_backward<kFused>(T, packet, lane, L, A, hg, hm);
        return;
    }
    const int64_t packet = logical_block(T.xcd_remap) * T.waves_per_group + wave;
    packet_backward<kFused>(T, packet, lane, L, A, nullptr, nullptr);
}

// Zero the accumulators (a fill kernel, so the call stays capturable).
__global__ void k_zero_f32(float *p, int64_t count) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0f;
}

// Chain rule from the per-Gaussian sums (g_rho, m, M) to the raw
// parameters. P = R L R^T with L = diag(s^-2): dL/dmu = P m,
// dL/dP = -M/2, so dL/ds_k = (r_k^T M r_k) / s_k^3 (r_k the k-th column of R)
// and dL/dR = -M R L. R(q) = (1 - 2|v|^2) I + 2 w [v]x + 2 v v^T for
// q = (w, v); for G = dL/dR:  dL/dw = 2 v . ax(G) and
// dL/dv = -4 tr(G) v + 2 w ax(G) + 2 (G + G^T) v, with
// ax(G) = (G21 - G12, G02 - G20, G10 - G01); finally the projection through
// q/|q|: dL/dq = (g - qh (qh . g)) / |q|.
__global__ __launch_bounds__(256) void k_epilogue(const float *__restrict__ mean,
                                                  const float *__restrict__ scale,
                                                  const float *__restrict__ quat,
                                                  const float *__restrict__ dens, int64_t n,
                                                  const uint32_t *__restrict__ order,
                                                  const float *__restrict__ acc, float *gmean,
                                                  float *gscale, float *gquat, float *gdens) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int64_t i = order[g];
    if (i >= n) return;
    double s[3], q[4], qq = 0.0;
    bool ok = isfinite(mean[i]) && isfinite(mean[n + i]) && isfinite(mean[2 * n + i]) &&
              isfinite(dens[i]);
    for (int k = 0; k < 3; ++k) {
        s[k] = scale[k * n + i];
        ok = ok && isfinite(s[k]) && s[k] > 0.0;
    }
    for (int k = 0; k < 4; ++k) {
        q[k] = quat[k * n + i];
        ok = ok && isfinite(q[k]);
        qq += q[k] * q[k];
    }
    ok = ok && qq > 0.0;
    if (!ok) {
        for (int k = 0; k < 3; ++k) gmean[k * n + i] = 0.0f, gscale[k * n + i] = 0.0f;
        for (int k = 0; k < 4; ++k) gquat[k * n + i] = 0.0f;
        gdens[i] = 0.0f;
        return;
    }
    double a[10];
    for (int k = 0; k < 10; ++k) a[k] = acc[k * n + g];
    const double qn = sqrt(qq);
    const double w = q[0] / qn, v[3] = {q[1] / qn, q[2] / qn, q[3] / qn};
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double R[3][3];
    const double cx[3][3] = {{0.0, -v[2], v[1]}, {v[2], 0.0, -v[0]}, {-v[1], v[0], 0.0}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            R[r][c] = (r == c ? 1.0 - 2.0 * vv : 0.0) + 2.0 * w * cx[r][c] + 2.0 * v[r] * v[c];
    const double lam[3] = {1.0 / (s[0] * s[0]), 1.0 / (s[1] * s[1]), 1.0 / (s[2] * s[2])};
    const double m[3] = {a[1], a[2], a[3]};
    const double M[3][3] = {{a[4], a[7], a[8]}, {a[7], a[5], a[9]}, {a[8], a[9], a[6]}};
    // dL/dmu = P m = R L R^T m
    double Rtm[3];
    for (int k = 0; k < 3; ++k) Rtm[k] = lam[k] * (R[0][k] * m[0] + R[1][k] * m[1] + R[2][k] * m[2]);
    for (int r = 0; r < 3; ++r) gmean[r * n + i] = float(R[r][0] * Rtm[0] + R[r][1] * Rtm[1] + R[r][2] * Rtm[2]);
    // M R (columns), then dL/ds and dL/dR
    double MR[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) MR[r][c] = M[r][0] * R[0][c] + M[r][1] * R[1][c] + M[r][2] * R[2][c];
    for (int k = 0; k < 3; ++k) {
        const double rMr = R[0][k] * MR[0][k] + R[1][k] * MR[1][k] + R[2][k] * MR[2][k];
        gscale[k * n + i] = float(rMr / (s[k] * s[k] * s[k]));
    }
    double G[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) G[r][c] = -MR[r][c] * lam[c];
    const double axg[3] = {G[2][1] - G[1][2], G[0][2] - G[2][0], G[1][0] - G[0][1]};
    const double tr = G[0][0] + G[1][1] + G[2][2];
    double gq[4];
    gq[0] = 2.0 * (v[0] * axg[0] + v[1] * axg[1] + v[2] * axg[2]);
    for (int k = 0; k < 3; ++k) {
        const double Gv = G[k][0] * v[0] + G[k][1] * v[1] + G[k][2] * v[2];
        const double GTv = G[0][k] * v[0] + G[1][k] * v[1] + G[2][k] * v[2];
        gq[1 + k] = -4.0 * tr * v[k] + 2.0 * w * axg[k] + 2.0 * (Gv + GTv);
    }
    const double qh[4] = {w, v[0], v[1], v[2]};
    const double dot = gq[0] * qh[0] + gq[1] * qh[1] + gq[2] * qh[2] + gq[3] * qh[3];
    for (int k = 0; k < 4; ++k) gquat[k * n + i] = float((gq[k] - qh[k] * dot) / qn);
    gdens[i] = float(a[0]);
}

// ---------------------------------------------------------------------------
// host drivers
// ---------------------------------------------------------------------------

static void finish_table(LaunchTable &T, const LaunchShape &shape) {
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
}

// Workgroups of a launch: one wave per packet, or the persistent count.
static unsigned launch_groups(const LaunchTable &T, const LaunchShape &shape) {
    if (shape.work_counter) return unsigned(shape.persistent_groups);
    return unsigned((T.n_packets + shape.waves - 1) / shape.waves);
}

__global__ void k_zero_u32(uint32_t *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}

hipError_t enqueue_forward(LaunchTable &T, const LaunchShape &shape, hipStream_t st, uint64_t *stats) {
    finish_table(T, shape);
    if (T.n_packets == 0) return hipSuccess;
    if (shape.work_counter) k_zero_u32<<<1, 64, 0, st>>>(shape.work_counter);
    const unsigned groups = launch_groups(T, shape);
    const int waves = shape.waves;
    const size_t lds = T.traversal == 1 ? 0 : sizeof(uint32_t) * kWideStack * size_t(waves);
    if (stats)
        k_forward<true><<<dim3(groups), dim3(64 * waves), lds, st>>>(T, stats);
    else
        k_forward<false><<<dim3(groups), dim3(64 * waves), lds, st>>>(T, nullptr);
    return hipGetLastError();
}

hipError_t enqueue_backward(LaunchTable &T, const BwdArgs &A, const gr_scene &sc, const uint32_t *order,
                            float *gmean, float *gscale, float *gquat, float *gdens,
                            const LaunchShape &shape, uint32_t *hit_g, uint64_t *hit_m,
                            hipStream_t st) {
    finish_table(T, shape);
    const bool lists = !A.grad_out && shape.work_counter && shape.hit_cap > 0 && hit_g && hit_m;
    T.hit_cap = lists ? shape.hit_cap : 0;
    T.hit_g = lists ? hit_g : nullptr;
    T.hit_m = lists ? hit_m : nullptr;
    const int64_t n = sc.n;
    if (n > 0) {
        const int64_t cnt = 10 * n;
        k_zero_f32<<<unsigned((cnt + 255) / 256), 256, 0, st>>>(A.acc, cnt);
    }
    if (T.n_packets > 0) {
        if (shape.work_counter) k_zero_u32<<<1, 64, 0, st>>>(shape.work_counter);
        const unsigned groups = launch_groups(T, shape);
        const int waves = shape.waves;
        if (A.grad_out)
            k_backward<false><<<dim3(groups), dim3(64 * waves), sizeof(WaveLdsPlain) * size_t(waves), st>>>(T, A);
        else
            k_backward<true><<<dim3(groups), dim3(64 * waves), sizeof(WaveLdsFused) * size_t(waves), st>>>(T, A);
    }
    if (n > 0)
        k_epilogue<<<unsigned((n + 255) / 256), 256, 0, st>>>(sc.mean, sc.scale, sc.quat, sc.density,
                                                              n, order, A.acc, gmean, gscale, gquat,
                                                              gdens);
    return hipGetLastError();
}

}  // namespace gr
