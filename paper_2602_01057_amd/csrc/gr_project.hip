// Ray-packet projection kernels: forward (Eq. 12 with the kappa cutoff),
// backward (gradient of a per-ray loss) and the fused forward -> loss ->
// backward pass.
//
// One wave64 owns one packet of 64 consecutive rays (one lane per ray):
//  1. the rays' bounding "beam" is built once per packet: a frame (a, e1, e2)
//     from the first ray's direction, and per-ray intercepts X and slopes S of
//     every line x(z) = X + z S in that frame, reduced to [min, max] ranges
//     with DPP;
//  2. the wave walks the 64-wide box hierarchy over the Morton-ordered leaves
//     (64 child boxes tested against the beam per wave step, pending nodes on
//     a per-wave LDS stack), or the binary LBVH with per-ray slab tests;
//  3. at a leaf, up to 64 Gaussians are tested lane-parallel against the beam
//     (support widths of each kappa ellipsoid along a, e1, e2), giving a
//     64-bit candidate mask;
//  4. for each candidate the 80-byte Gaussian record is fetched with scalar
//     loads and every lane evaluates the closed form for its ray.
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
// (the last by the envelope theorem on D = min_t). Per Gaussian the backward
// sums, in FP32,
//   g_rho = sum w T/rho, m = sum w T p, M = sum w T (p p^T + d d^T / A)
// (10 floats) and adds them to the Gaussian's accumulators with float
// atomics; k_epilogue maps them to mean, scale and quaternion gradients. The
// fused pass records each packet's (Gaussian, ray mask) hit list in its forward
// half and replays it with the pairs spread evenly over the lanes; with dL/dI
// given, or for a list that outgrew its region, the backward re-traverses and
// runs Gaussian-major (candidates one per lane, each looping over the packet's
// weighted rays).
#include <type_traits>

#include "gr_trace.h"

namespace gr {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Forward sum over one leaf's candidate Gaussians (mask), two records per
// step. The compiler issues each record's scalar loads at its first use (the
// density's inside the branch of the lanes within the cutoff); the 8 waves per
// SIMD of k_forward hide those latencies. Holding both records before the
// first evaluation (hold_records, as the recording loop of the fused pass
// does) ran this kernel 4% slower: more scalar registers spill at 8 waves.
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

// Eq. 7 for one pair in FP32 from the compact record (the forward's FP32
// precision mode). The offset o - mu is kept exactly as hi + lo (TwoSum), the
// origin slides along the line to the point nearest mu (t0 = -hi.d / d.d;
// sliding does not change the integral), and with u = W delta', v = W d
// (P = W^T W): A = v.v, B = u.v and D = |u - (B/A) v|^2, which loses far less
// to cancellation than C - B^2/A. r = 1/sqrt(A).
__device__ inline void pair_core32(const GaussRec32 &G, const Ray &R, float inv_dd, float &D, float &r) {
    float hi[3], lo[3];
    for (int k = 0; k < 3; ++k) {
        const float a = R.o[k], b = -G.mu[k];
        const float s = a + b;
        const float bv = s - a;
        lo[k] = (a - (s - bv)) + (b - bv);
        hi[k] = s;
    }
    const float t0 = -(hi[0] * R.d[0] + hi[1] * R.d[1] + hi[2] * R.d[2]) * inv_dd;
    float dl[3];
    for (int k = 0; k < 3; ++k) dl[k] = fmaf(t0, R.d[k], hi[k]) + lo[k];
    float u[3], v[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = G.W[3 * a] * dl[0] + G.W[3 * a + 1] * dl[1] + G.W[3 * a + 2] * dl[2];
        v[a] = G.W[3 * a] * R.d[0] + G.W[3 * a + 1] * R.d[1] + G.W[3 * a + 2] * R.d[2];
    }
    const float A = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const float B = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    r = __builtin_amdgcn_rsqf(A);
    const float tB = B * (r * r);
    const float p0 = fmaf(-tB, v[0], u[0]), p1 = fmaf(-tB, v[1], u[1]), p2 = fmaf(-tB, v[2], u[2]);
    D = p0 * p0 + p1 * p1 + p2 * p2;
}

// leaf_forward in the FP32 precision mode (compact records, two per step).
template <bool kStats>
__device__ inline void leaf_forward32(const SceneView &S, const Ray &R, float inv_dd, int64_t start,
                                      uint64_t mask, float k2, bool active, double &acc, uint32_t &n_inc,
                                      uint32_t &n_hitc) {
    while (mask) {
        const int j0 = __builtin_ctzll(mask);
        mask &= mask - 1;
        const bool two = mask != 0;
        const int j1 = two ? __builtin_ctzll(mask) : j0;
        if (two) mask &= mask - 1;
        const GaussRec32 *rec32 = rec32_of(S);
        const GaussRec32 G0 = sload(rec32, start + j0);
        const GaussRec32 G1 = sload(rec32, start + j1);
        float D, r;
        pair_core32(G0, R, inv_dd, D, r);
        if (kStats) n_hitc += ballot(active && D <= k2) != 0 ? 1u : 0u;
        if (D <= k2) {
            acc += double(G0.rho_c * r * gauss_exp(D));
            if (kStats) n_inc += active ? 1u : 0u;
        }
        if (two) {
            pair_core32(G1, R, inv_dd, D, r);
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
// kCompact selects the FP32 precision mode.
template <bool kStats, bool kCompact>
__device__ inline void packet_forward(const LaunchTable &T, int64_t packet, int lane, uint32_t *stack,
                                      uint64_t *stats) {
    PacketRef P;
    if (!locate_packet(T, packet, lane, P)) return;
    const Segment &sg = T.segs[P.seg];
    const SceneView &S = T.scenes[sg.scene];
    float *out = sg.out;
    Ray R;
    load_ray(sg.ro, sg.rd, sg.stride, P.ray, R);
    Beam B;
    build_beam(R, B);
    double acc = 0.0;
    const float k2 = S.kappa2;
    uint32_t n_inc = 0, n_cand = 0, n_leaf = 0, n_hitc = 0;
    const float inv_dd = kCompact ? 1.0f / (R.d[0] * R.d[0] + R.d[1] * R.d[1] + R.d[2] * R.d[2]) : 0.0f;
    traverse_any(T.traversal, S, R, B, P.active, lane, stack, [&](int l) {
        int64_t start;
        const uint64_t mask = leaf_candidates(S, B, l, lane, start);
        if (kStats) {
            ++n_leaf;
            n_cand += __builtin_popcountll(mask);
        }
        if constexpr (kCompact)
            leaf_forward32<kStats>(S, R, inv_dd, start, mask, k2, P.active, acc, n_inc, n_hitc);
        else
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

// 8 waves per SIMD (at most 64 VGPRs; the traversal state spills a few
// registers, the pair loop none): the forward waits on its records' loads,
// and more waves hide that latency (8 waves ran the 500k workload 6% faster
// than the 7 that its 71 VGPRs allow unforced).
template <bool kStats, bool kCompact>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_forward(
    LaunchTable T, uint64_t *stats) {
    extern __shared__ uint32_t fwd_stack[];  // kWideStack entries per wave
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    uint32_t *stack = fwd_stack + wave * kWideStack;
    if (T.work_counter) {
        // persistent: waves pull packets until the table is exhausted
        for (int64_t packet = next_packet(T.work_counter, lane); packet < T.n_packets;
             packet = next_packet(T.work_counter, lane))
            packet_forward<kStats, kCompact>(T, packet, lane, stack, stats);
        return;
    }
    const int64_t packet = logical_block(T.xcd_remap) * T.waves_per_group + wave;
    packet_forward<kStats, kCompact>(T, packet, lane, stack, stats);
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
// res[k][entry]). 64 entries take 8.5 KB per wave, so the 160 KB of a compute
// unit hold 18 waves' windows, against the 20 that the fused kernel's
// registers allow.
constexpr int kWin = 64;
constexpr int kWinLog2 = 6;  // search steps: 2^6 >= kWin
struct HitWindow {
    union {
        GaussRec rec[kWin];
        float part[10][kWin];  // lanes' closing sums, once the window's pairs are done
    };
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

// v_writelane_b32: returns old with lane `lane` replaced by the wave-uniform
// value (the LLVM intrinsic; this compiler has no builtin for it).
__device__ int lane_write(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

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
    uint32_t bg;  // lane i holds pending entry i: Gaussian index,
    uint32_t blo; // low and
    uint32_t bhi; // high half of its ray mask

    __device__ void flush(int lane) {
        if (nbuf == 0) return;
        if (n + nbuf <= cap) {
            if (lane < nbuf) {
                g[n + lane] = bg;
                m[n + lane] = (uint64_t(bhi) << 32) | blo;
            }
            n += nbuf;
        } else {
            overflow = true;
        }
        nbuf = 0;
    }
    // Appends (gi, mask); both are wave-uniform and mask is non-zero. The
    // entry goes into lane nbuf of the pending registers by lane writes.
    __device__ void record(int lane, int64_t gi, uint64_t mask) {
        if (overflow) return;
        bg = lane_write(int(uint32_t(gi)), nbuf, int(bg));
        blo = lane_write(int(uint32_t(mask)), nbuf, int(blo));
        bhi = lane_write(int(uint32_t(mask >> 32)), nbuf, int(bhi));
        if (++nbuf == 64) flush(lane);
    }
};

// Forward sum over one leaf's candidates (as leaf_forward), also recording the
// packet's hit list.
__device__ inline void leaf_forward_hits(const SceneView &S, const Ray &R, int64_t start, uint64_t mask,
                                         float k2, bool active, double &acc, HitList &H, int lane) {
    // A lane past the last ray compares against a negative cutoff, which no
    // D >= 0 passes: the ballot is then one compare.
    const float k2a = active ? k2 : -1.0f;
    while (mask) {
        const int j0 = __builtin_ctzll(mask);
        mask &= mask - 1;
        const bool two = mask != 0;
        const int j1 = two ? __builtin_ctzll(mask) : j0;
        if (two) mask &= mask - 1;
        const GaussRec G0 = sload(S.rec, start + j0);
        const GaussRec G1 = sload(S.rec, start + j1);
        hold_records(G0, G1);
        PairCore c;
        float D, r;
        pair_core(G0.mu, G0.P, R.o64, R.d64, R.dd, c);
        pair_D(c, D, r);
        const uint64_t h0 = __builtin_amdgcn_ballot_w64(D <= k2a);
        if (h0) {
            if (D <= k2a) {
                asm volatile("");  // keeps this a branch: if-converted, every lane pays for the exp
                acc += double(G0.rho_c * r * gauss_exp(D));
            }
            H.record(lane, start + j0, h0);
        }
        if (two) {
            pair_core(G1.mu, G1.P, R.o64, R.d64, R.dd, c);
            pair_D(c, D, r);
            const uint64_t h1 = __builtin_amdgcn_ballot_w64(D <= k2a);
            if (h1) {
                if (D <= k2a) {
                    asm volatile("");
                    acc += double(G1.rho_c * r * gauss_exp(D));
                }
                H.record(lane, start + j1, h1);
            }
        }
    }
}

// Backward half from a recorded hit list, in windows of kWin entries. The T
// included pairs of a window are split evenly over the lanes (lane k takes
// pairs [k s, k s + s) of the window's pairs in list order, s = ceil(T / 64)),
// so every lane is busy however unequal the entries' ray counts are. A lane
// that moves on from an entry stores its sums into the window's LDS slot for
// it; the sums for the entry it is in when its range ends are added per run
// of lanes ending in that entry, with no LDS atomics. At the end of the
// window lane j adds entry j's sums to the global
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
                // Entry e ends inside this lane's range, so no other lane
                // leaves it inside the loop: the lanes that also hold part of
                // it hold its start and add their sums after the loop. Its
                // slot is still zero here, and a plain store replaces the
                // LDS float atomic.
                for (int k = 0; k < 10; ++k) {
                    W.res[k][e] = c[k];
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
        close_window<kWin>(W.part, W.res, c, left > 0 ? e : -1, lane);
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
    const SceneView &S = T.scenes[sg.scene];
    Ray R;
    load_ray(sg.ro, sg.rd, sg.stride, P.ray, R);
    Beam B;
    build_beam(R, B);
    const float k2 = S.kappa2;
    if constexpr (kFused) {
        float *acc = sg.acc;
        bool listed = false;  // the forward half recorded a complete hit list
        int n_ent = 0;
        double sum = 0.0;
        if (T.hit_cap > 0 && hit_g) {
            HitList H{hit_g, hit_m, T.hit_cap, 0, 0, false, 0u, 0u, 0u};
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
            w = loss_weight(sg.loss_kind, I, sg.target[P.out], sg.background, term);
            if (sg.out) sg.out[P.out] = I;
        }
        if (sg.loss) {
            for (int off = 32; off >= 1; off >>= 1) term += __shfl_xor(term, off);
            if (lane == 0) atomicAdd(sg.loss, term);
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
        float *acc = A.acc;
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

// 5 waves per SIMD (at most 96 VGPRs, against the 126 the fused form takes
// unforced; a few registers spill): the forward half of the fused pass waits
// on its records' loads, and the extra wave hides part of that latency
// (persistent launches default to 20 waves per compute unit to match; LDS
// holds 18 windows per compute unit, and later workgroups start as earlier
// ones finish).
template <bool kFused>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5))) void k_backward(LaunchTable T, BwdArgs A) {
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
    if (T.precision == 1) {
        if (stats)
            k_forward<true, true><<<dim3(groups), dim3(64 * waves), lds, st>>>(T, stats);
        else
            k_forward<false, true><<<dim3(groups), dim3(64 * waves), lds, st>>>(T, nullptr);
    } else {
        if (stats)
            k_forward<true, false><<<dim3(groups), dim3(64 * waves), lds, st>>>(T, stats);
        else
            k_forward<false, false><<<dim3(groups), dim3(64 * waves), lds, st>>>(T, nullptr);
    }
    return hipGetLastError();
}

static void launch_backward(LaunchTable &T, const BwdArgs &A, const LaunchShape &shape, uint32_t *hit_g,
                            uint64_t *hit_m, hipStream_t st) {
    finish_table(T, shape);
    const bool lists = !A.grad_out && shape.work_counter && shape.hit_cap > 0 && hit_g && hit_m;
    T.hit_cap = lists ? shape.hit_cap : 0;
    T.hit_g = lists ? hit_g : nullptr;
    T.hit_m = lists ? hit_m : nullptr;
    if (T.n_packets == 0) return;
    if (shape.work_counter) k_zero_u32<<<1, 64, 0, st>>>(shape.work_counter);
    const unsigned groups = launch_groups(T, shape);
    const int waves = shape.waves;
    if (A.grad_out)
        k_backward<false><<<dim3(groups), dim3(64 * waves), sizeof(WaveLdsPlain) * size_t(waves), st>>>(T, A);
    else
        k_backward<true><<<dim3(groups), dim3(64 * waves), sizeof(WaveLdsFused) * size_t(waves), st>>>(T, A);
}

hipError_t enqueue_backward(LaunchTable &T, const BwdArgs &A, const gr_scene &sc, const uint32_t *order,
                            float *gmean, float *gscale, float *gquat, float *gdens,
                            const LaunchShape &shape, uint32_t *hit_g, uint64_t *hit_m,
                            hipStream_t st) {
    enqueue_zero_f32(A.acc, 10 * sc.n, st);
    launch_backward(T, A, shape, hit_g, hit_m, st);
    enqueue_epilogue(sc, order, A.acc, gmean, gscale, gquat, gdens, st);
    return hipGetLastError();
}

hipError_t enqueue_fused_segments(LaunchTable &T, const LaunchShape &shape, uint32_t *hit_g, uint64_t *hit_m,
                                  hipStream_t st) {
    BwdArgs A{nullptr, nullptr};
    launch_backward(T, A, shape, hit_g, hit_m, st);
    return hipGetLastError();
}

void enqueue_zero_u32(uint32_t *p, hipStream_t st) { k_zero_u32<<<1, 64, 0, st>>>(p); }

void enqueue_zero_f32(float *p, int64_t count, hipStream_t st) {
    if (count > 0) k_zero_f32<<<unsigned((count + 255) / 256), 256, 0, st>>>(p, count);
}

void enqueue_epilogue(const gr_scene &sc, const uint32_t *order, const float *acc, float *gmean, float *gscale,
                      float *gquat, float *gdens, hipStream_t st) {
    const int64_t n = sc.n;
    if (n > 0)
        k_epilogue<<<unsigned((n + 255) / 256), 256, 0, st>>>(sc.mean, sc.scale, sc.quat, sc.density, n, order,
                                                              acc, gmean, gscale, gquat, gdens);
}

}  // namespace gr
