// Device building blocks shared by the projection kernels (plain, fused and
// time-of-flight): wave helpers, the per-lane ray and per-wave beam, the FP64
// pair core of Eq. 7, the binary and 64-wide traversals with beam tests, and
// packet location in a launch table. Everything here is inline device code.
#pragma once

#include <float.h>
#include <math.h>

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

// Closing step of a replay window whose pairs are split over the lanes in
// consecutive ranges (the hit-list and TOF replays). A lane that moved on from
// an entry inside its range has stored that entry's sums already; what is left
// is each lane's sums c for the entry fe its range ends in (fe < 0: the lane
// had no pairs). Lanes ending in the same entry are consecutive, since their
// last pairs increase with the lane, so the first lane of each run adds the
// run's sums to res[.][fe] with one read-modify-write and no LDS atomics;
// part (10 x 64 floats, free by now) carries the other lanes' sums.
template <int kSlots>
__device__ inline void close_window(float (*part)[64], float (*res)[kSlots], float c[10], int fe, int lane) {
    const int fe_prev = __shfl(fe, (lane + 63) & 63, 64);
    const bool head = fe >= 0 && (lane == 0 || fe_prev != fe);
    const uint64_t heads = ballot(head);
    const int n_closing = __builtin_popcountll(ballot(fe >= 0));  // a prefix of the lanes
    __builtin_amdgcn_wave_barrier();
    if (fe >= 0 && !head)
        for (int k = 0; k < 10; ++k) part[k][lane] = c[k];
    __builtin_amdgcn_wave_barrier();
    if (head) {
        const uint64_t later = lane < 63 ? heads >> (lane + 1) : 0ull;
        const int run_end = later ? lane + 1 + __builtin_ctzll(later) : n_closing;
        for (int l = lane + 1; l < run_end; ++l)
            for (int k = 0; k < 10; ++k) c[k] += part[k][l];
        for (int k = 0; k < 10; ++k) res[k][fe] += c[k];
    }
    __builtin_amdgcn_wave_barrier();
}

// Both records of a traversal step held in scalar registers before either is
// used, so that the step waits for memory once: the compiler otherwise issues
// each record's loads at its first use, and the density's inside the branch
// of the lanes within the cutoff, each followed by its own wait.
__device__ inline void hold_records(const GaussRec &a, const GaussRec &b) {
    asm volatile("" ::"s"(a.mu[0]), "s"(a.rho_c), "s"(b.mu[0]), "s"(b.rho_c));
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

// Next packet of a persistent launch: lane 0 takes a ticket from the work
// counter and the wave shares it.
__device__ inline int64_t next_packet(uint32_t *counter, int lane) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(counter, 1u);
    return int64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(t))));
}

}  // namespace gr
