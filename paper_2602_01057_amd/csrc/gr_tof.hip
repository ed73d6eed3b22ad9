// Time-of-flight PET projection with attenuation: the projector extensions
// the paper names as future work (Sec. 5), kept in closed form.
//
// Model. Bin b of ray r weighs the line by the TOF kernel
//   h_b(t) = (w / (sqrt(2 pi) sigma)) exp(-(t - tau_b)^2 / (2 sigma^2)),
//   tau_b  = c_r + (b - (n_bins - 1)/2) w,
// (w the bin spacing, c_r the ray's TOF centre) and the ray's attenuation
// factor a_r multiplies every bin. Along the ray a Gaussian is
// T sqrt(A/(2 pi)) exp(-A (t - t*)^2 / 2) with T its plain line integral
// (Eq. 11) and t* = -B/A, so its bin value is T times a 1D Gaussian of the bin
// centre:
//   I_b = a_r T g_b,  g_b = w / sqrt(2 pi s^2) exp(-(tau_b - t*)^2 / (2 s^2)),
//   s^2 = sigma^2 + 1/A.
// (Equal to the closed form with A' = A + 1/sigma^2, B' = B - tau_b/sigma^2,
// C' = C + tau_b^2/sigma^2; this factored form reuses the plain pair values
// and costs one exponential per bin.) Pairs count as in the projection,
// D <= kappa^2.
//
// Gradient. With W = sum_b v_b g_b over the ray's bin weights v_b = a_r
// dL/dI_b, F = T W depends on the Gaussian through T, t* and s^2. Using
// dt*/dmu = P d / A, dt*/dP = -sym(d p^T)/A, ds^2/dP = -d d^T / A^2 and the
// plain dT (p = delta + t* d):
//   dF/dmu = P (W T p + alpha d),
//   dF/dP  = -(1/2) [W T p p^T + alpha (d p^T + p d^T) + beta d d^T],
//   alpha  = T W_t / A,  beta = W T / A + 2 T W_s / A^2,
//   W_t = sum v_b g_b u_b / s^2,  W_s = sum v_b g_b (u_b^2/(2 s^4) - 1/(2 s^2)),
// u_b = tau_b - t*. These are the plain backward's ten sums (rho term,
// m = sum q, M = sum q p^T + v d^T with q = W T p + alpha d,
// v = alpha p + beta d), so the same epilogue maps them to the parameters.
// Without a TOF kernel W = a_r dL/dI and W_t = W_s = 0.
//
// Kernels: the packet traversal of the plain projector (one wave per 64
// rays). The forward keeps kBins FP64 accumulators per ray in its lane (bins
// guarded by n_bins) and queues its included pairs per lane, evaluating their
// bins once most lanes have one waiting. The backward takes the cutoff test for every candidate
// on all rays, records hit windows and replays them with the included pairs
// spread evenly over the lanes; the rays' bin weights sit in LDS.
#include <algorithm>
#include <type_traits>

#include "gr_trace.h"

namespace gr {

namespace {

constexpr double kLog2eD = 1.4426950408889634074;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

__device__ inline float ray_center(const TofArgs &A, int64_t ray) { return A.center ? A.center[ray] : 0.0f; }
__device__ inline float ray_atten(const TofArgs &A, int64_t ray) { return A.atten ? A.atten[ray] : 1.0f; }

// A ray as its lane holds it for the replay: the FP32 origin and direction
// (exact in FP64) and the TOF centre.
struct TofRayF {
    float o[3], d[3];
    float c;
};

// Ray i from the lane that holds it (ds_bpermute: every lane executes this).
__device__ inline TofRayF gather_tof_ray(const TofRayF &mine, int i) {
    const int a = i << 2;
    auto g = [&](float v) {
        return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(a, __builtin_bit_cast(int, v)));
    };
    TofRayF r;
    for (int k = 0; k < 3; ++k) {
        r.o[k] = g(mine.o[k]);
        r.d[k] = g(mine.d[k]);
    }
    r.c = g(mine.c);
    return r;
}

// Hit windows of the backward. The traversal takes the cutoff test
// D <= kappa^2 for every candidate on all of the packet's rays (one ray per
// lane) and records
// (Gaussian, 64-bit mask of the rays inside) for each candidate with at least
// one; lane q keeps the q-th pending entry in registers. A full window, or the
// end of the packet, is replayed: the entries' records go to LDS and the
// window's T included pairs are split evenly over the lanes (lane k takes
// pairs [k s, k s + s) in list order, s = ceil(T / 64)), so every lane
// evaluates an included pair at every step of the bin loop, however unequal
// the entries' ray counts are. Without the replay the bin loop would run at
// the traversal's lane utilisation (about a quarter on the PET workload).
constexpr int kTofWin = 32;
constexpr int kTofWinLog2 = 5;  // search steps: 2^5 >= kTofWin

// A window in LDS: the entries' records, their gradient sums (SoA), masks and
// inclusive prefix counts of their pairs.
struct TofWinB {
    union {
        GaussRec rec[kTofWin];
        float part[10][64];  // lanes' closing sums, once the window's pairs are done
    };
    float res[10][kTofWin];
    uint64_t m[kTofWin];
    int32_t incl[kTofWin];
    int32_t pad[kTofWin];
};

// Rows of per-bin values per wave: the bins padded to a multiple of four.
__host__ __device__ constexpr int tof_rows(int nw) { return (nw + 3) & ~3; }

// Per-wave LDS of the backward: the window, the traversal stack, and 64 floats
// per row of bin weights (one per line).
template <class Win>
__host__ __device__ constexpr size_t tof_wave_bytes(int nw) {
    return sizeof(Win) + sizeof(uint32_t) * kWideStack + sizeof(float) * 64 * size_t(nw);
}

template <class Win>
struct TofWave {
    Win *win;
    uint32_t *stack;
    float *bins;  // [nw][64]
};

template <class Win>
__device__ inline TofWave<Win> tof_wave(unsigned char *base, int wave, int nw) {
    unsigned char *p = base + size_t(wave) * tof_wave_bytes<Win>(nw);
    TofWave<Win> w;
    w.win = reinterpret_cast<Win *>(p);
    w.stack = reinterpret_cast<uint32_t *>(p + sizeof(Win));
    w.bins = reinterpret_cast<float *>(p + sizeof(Win) + sizeof(uint32_t) * kWideStack);
    return w;
}

// Pending window entries (count wave-uniform; lane q holds entry q).
struct TofPending {
    int n;
    uint32_t g;
    uint64_t m;
    __device__ void put(int lane, int64_t gi, uint64_t mask) {
        if (lane == n) {
            g = uint32_t(gi);
            m = mask;
        }
        ++n;
    }
};

// This lane's share of a window: entry e with the rays still to do in m,
// `left` pairs, `s` steps for the wave.
struct TofShare {
    int e;
    uint64_t m;
    int left;
    int s;
};

// Stages the window's nq pending entries (all non-empty) in LDS and splits
// its pairs over the lanes.
template <class Win>
__device__ inline TofShare stage_window(const SceneView &S, Win &W, const TofPending &pe, int lane) {
    const int nq = pe.n;
    const bool own = lane < nq;
    const int cq = own ? __builtin_popcountll(pe.m) : 0;
    const int incl = wave_incl_scan(cq);
    const int T = __builtin_amdgcn_readlane(incl, 63);
    if (own) {
        W.rec[lane] = S.rec[pe.g];
        W.m[lane] = pe.m;
        W.incl[lane] = incl;
    }
    __builtin_amdgcn_wave_barrier();
    TofShare sh;
    sh.s = (T + 63) >> 6;
    const int p = lane * sh.s;
    sh.left = max(0, min(sh.s, T - p));
    // first entry whose inclusive count exceeds p (binary search over lanes)
    const int inclq = own ? incl : T;
    int lo = 0, hi = kTofWin - 1;
    for (int step = 0; step < kTofWinLog2; ++step) {
        const int mid = (lo + hi) >> 1;
        const int v = __shfl(inclq, mid, 64);
        if (v > p) hi = mid; else lo = mid + 1;
    }
    sh.e = sh.left > 0 ? lo : 0;
    uint64_t m = W.m[sh.e];
    // skip the entry's first (p - exclusive prefix) rays
    if (sh.left > 0) m = drop_low_bits(m, p - (W.incl[sh.e] - __builtin_popcountll(m)));
    sh.m = m;
    return sh;
}

// Bin geometry of a TOF launch: bin b's centre minus t* is
// (c - half) + b w + B/A with half = (n_bins - 1) w / 2.
struct TofBins {
    int nb;
    double half, wd;
    float kw;  // w / sqrt(2 pi)
    float sigma2;
};

__device__ inline TofBins tof_bins(const TofArgs &A) {
    TofBins b;
    b.nb = A.n_bins;
    b.half = 0.5 * double(A.n_bins - 1) * double(A.width);
    b.wd = A.width;
    b.kw = A.width * kInvSqrt2Pi;
    b.sigma2 = A.sigma2;
    return b;
}

// 1/x in FP64 from the FP32 reciprocal and one Newton step: the relative
// error squares from ~1e-7 to ~1e-14. x is s^2 = sigma^2 + 1/A >= 1e-24 (the
// API refuses sigma < 1e-12), inside FP32's normal range; above it the FP32
// reciprocal goes to 0 and so does the exact exponent q u^2 for any bin
// offset u a scanner has.
__device__ inline double rcp_newton(double x) {
    const double r = double(__builtin_amdgcn_rcpf(float(x)));
    return fma(r, fma(-x, r, 1.0), r);
}

// 2^x in FP64 for |x| <= 1020: x = n + f with n = rint(x) and |f| <= 1/2,
// 2^f from the Taylor series of e^y at y = f ln 2 to degree 10 (the truncated
// term is below 3e-13 relative), scaled by 2^n exactly.
__device__ inline double exp2_series(double x) {
    const double n = rint(x);
    const double y = (x - n) * 0.69314718055994530942;
    double p = 1.0 / 3628800.0;
    p = fma(p, y, 1.0 / 362880.0);
    p = fma(p, y, 1.0 / 40320.0);
    p = fma(p, y, 1.0 / 5040.0);
    p = fma(p, y, 1.0 / 720.0);
    p = fma(p, y, 1.0 / 120.0);
    p = fma(p, y, 1.0 / 24.0);
    p = fma(p, y, 1.0 / 6.0);
    p = fma(p, y, 0.5);
    p = fma(p, y, 1.0);
    p = fma(p, y, 1.0);
    return ldexp(p, int(n));
}

// A pair's bin values along the ray: bin b is 2^(e_b) with
// e_b = q (u0 + b w)^2, q = -log2(e) / (2 s^2) (the TOF Gaussian of the bin
// centre's offset u0 + b w from t*). The exponents are stepped by second
// differences in FP64 (e += de, de += dde; 25 steps round to ~1e-13).
//   - Fast form: the values themselves step by products, g_{b+1} = g_b r_b and
//     r_{b+1} = r_b K with g_0 = 2^e_0, r_0 = 2^de_0, K = 2^dde from
//     exp2_series: three exponentials per pair instead of one per bin, and
//     relative errors of ~1e-13 b^2 (FP64). It needs e_0, de_0 and dde inside
//     FP64's exponent range; the values then stay normal until they fall below
//     2^-1000, far under FP32's range.
//   - Otherwise (narrow kernels far from bin 0) each bin takes exp2 of its FP64
//     exponent rounded once to FP32.
// The empty asm statements tie each step to the bin's sum, so that the
// compiler keeps the chain in step with the bins instead of hoisting all kBins
// values ahead into registers.
struct BinChain {
    double e, de, dde;
    __device__ BinChain(double q, double u0, double w)
        : e(q * u0 * u0), de(q * fma(2.0, u0, w) * w), dde(2.0 * q * w * w) {}
    __device__ bool fast() const { return e > -1000.0 && de < 1000.0 && dde > -1000.0; }
    // fast form: g = 2^e_0, r = 2^de_0, K = 2^dde (unscaled, so that g_0 is
    // normal in FP64 whatever the pair's amplitude)
    __device__ void start(double &g, double &r, double &K) const {
        g = exp2_series(e);
        r = exp2_series(de);
        K = exp2_series(dde);
    }
    template <class Acc>
    __device__ static void step(double &g, double &r, double K, Acc &t) {
        g *= r;
        r *= K;
        asm volatile("" : "+v"(g), "+v"(r), "+v"(t));
    }
    // per-bin form: exp2 of this bin's exponent, then a step
    template <class Acc>
    __device__ float next(Acc &t) {
        const float x = float(e);
        e += de;
        de += dde;
        asm volatile("" : "+v"(e), "+v"(de), "+v"(t));
        return __builtin_amdgcn_exp2f(x);
    }
};

// Pairs of the TOF forward waiting for their bins, per lane (= line) in LDS:
// 1/A, B/A (= -t*) and the pair's line integral T. A lane queues its
// included pairs while the traversal goes on and the wave evaluates the bins
// once most lanes have one waiting, so that the bin loop runs with most lanes
// busy instead of only those inside the cutoff of the current candidate (a
// quarter on the PET workload). Each lane takes its pairs in the order it
// queued them, so the sums are the same as evaluating them in place.
constexpr int kTofQ = 8;       // pending pairs per lane (a power of 2)
constexpr int kTofReady = 48;  // a bin step once this many lanes have one
struct TofQueue {
    double ra[kTofQ][64];
    double tn[kTofQ][64];
    float tv[kTofQ][64];
};

// f(integral_constant<int, b>) for b = B, B + 1, ... below N, in groups of
// four with an early exit before a group that starts at or past n: an
// unrolled loop whose bin index is a compile-time constant, so that per-bin
// registers stay registers (the loop unroller gives up on the bin loops once
// they sit inside the forward's queue service loop). The bins of the last
// group past n go to sums that are never read; one exit test per group keeps
// the compiler from holding a test mask per bin (spilled to VGPR lanes and
// read back with two instructions per bin).
template <int B, int N, class F>
__device__ __attribute__((always_inline)) inline void bins_until(int n, F &&f) {
    if constexpr (B < N) {
        if (B >= n) return;
        f(std::integral_constant<int, B>{});
        if constexpr (B + 1 < N) f(std::integral_constant<int, B + 1>{});
        if constexpr (B + 2 < N) f(std::integral_constant<int, B + 2>{});
        if constexpr (B + 3 < N) f(std::integral_constant<int, B + 3>{});
        bins_until<B + 4, N>(n, f);
    }
}

// The bins of one pair added to the line's FP64 sums: t* = -tn, s^2 =
// sigma^2 + 1/A, and the chain of bin values (3 FP64 instructions per bin).
template <int kBins>
__device__ __attribute__((always_inline)) inline void add_pair_bins(const TofBins &tb, double c0, double ra,
                                                                    double tn, float Tv, double acc[kBins]) {
    const double u0 = c0 + tn;  // tau_0 - t*
    const double s2d = double(tb.sigma2) + ra;
    // the exponents in FP64: deep in the kernel's tail (|exponent| ~ 100) an
    // FP32 chain would cost ~1e-5
    BinChain ch(-0.5 * kLog2eD * rcp_newton(s2d), u0, tb.wd);
    const float Tg = Tv * tb.kw * __builtin_amdgcn_rsqf(float(s2d));
    if (ch.fast()) {
        double g, rb, K;
        ch.start(g, rb, K);
        const double Tgd = Tg;
        bins_until<0, kBins>(tb.nb, [&](auto b) {
            acc[b] = fma(Tgd, g, acc[b]);
            BinChain::step(g, rb, K, acc[b]);
        });
    } else {
        // (tied to the previous bin's sum, which is done by then)
        bins_until<0, kBins>(tb.nb, [&](auto b) { acc[b] += double(Tg * ch.next(acc[b > 0 ? b - 1 : 0])); });
    }
}

// One packet of the TOF forward: every lane takes the cutoff test of each
// candidate for its line; the lanes inside it queue the pair for its bins.
template <int kBins>
__device__ inline void packet_forward_tof(const LaunchTable &T, const TofArgs &A, int64_t packet, int lane,
                                          uint32_t *stack, TofQueue &Q) {
    PacketRef P;
    if (!locate_packet(T, packet, lane, P)) return;
    const Segment &sg = T.segs[P.seg];
    const SceneView &S = T.scenes[sg.scene];
    Ray R;
    load_ray(sg.ro, sg.rd, sg.stride, P.ray, R);
    Beam B;
    build_beam(R, B);
    const float k2 = S.kappa2;
    const TofBins tb = tof_bins(A);
    const bool tof = tb.nb > 0;
    const double c0 = double(ray_center(A, P.ray)) - tb.half;
    double acc[kBins];
#pragma unroll
    for (int b = 0; b < kBins; ++b) acc[b] = 0.0;
    int head = 0, cnt = 0;  // this lane's queue
    auto bin_step = [&]() __attribute__((always_inline)) {
        if (cnt > 0) {
            const double ra = Q.ra[head][lane], tn = Q.tn[head][lane];
            const float Tv = Q.tv[head][lane];
            head = (head + 1) & (kTofQ - 1);
            --cnt;
            add_pair_bins<kBins>(tb, c0, ra, tn, Tv, acc);
        }
    };
    // the cutoff test of one candidate; a pair inside it is queued
    auto pair_in = [&](const GaussRec &G) __attribute__((always_inline)) {
        PairCore c;
        float D, r;
        pair_core(G.mu, G.P, R.o64, R.d64, R.dd, c);
        pair_D(c, D, r);
        if (D <= k2) {
            const float Tv = G.rho_c * r * gauss_exp(D);
            if (!tof) {
                acc[0] += double(Tv);
            } else {
                // 1/A from the FP32 r^2 and one Newton step, t* = -B/A in FP64
                double ra = double(r * r);
                ra = fma(ra, fma(-c.A, ra, 1.0), ra);
                const int slot = (head + cnt) & (kTofQ - 1);
                Q.ra[slot][lane] = ra;
                Q.tn[slot][lane] = c.B * ra;
                Q.tv[slot][lane] = Tv;
                ++cnt;
            }
        }
    };
    traverse_any(T.traversal, S, R, B, P.active, lane, stack, [&](int l) {
        int64_t start;
        uint64_t mask = leaf_candidates(S, B, l, lane, start);
        // two candidates per step (their records load together)
        while (mask) {
            const int j0 = __builtin_ctzll(mask);
            mask &= mask - 1;
            const bool two = mask != 0;
            const int j1 = two ? __builtin_ctzll(mask) : j0;
            if (two) mask &= mask - 1;
            const GaussRec G0 = sload(S.rec, start + j0);
            const GaussRec G1 = sload(S.rec, start + j1);
            hold_records(G0, G1);
            pair_in(G0);
            if (two) pair_in(G1);
            // bin steps while a queue lacks room for the next step's two pairs
            // or most lanes have a pair waiting
            if (tof) {
                for (;;) {
                    const bool full = ballot(cnt > kTofQ - 2) != 0;
                    if (!full && __builtin_popcountll(ballot(cnt > 0)) < kTofReady) break;
                    bin_step();
                }
            }
        }
    });
    while (ballot(cnt > 0)) bin_step();
    if (P.active) {
        const float a = ray_atten(A, P.ray);
        const int nout = tof ? tb.nb : 1;
#pragma unroll
        for (int b = 0; b < kBins; ++b)
            if (b < nout) A.out[int64_t(b) * A.n_rays + P.out] = float(double(a) * acc[b]);
    }
}

template <int kBins>
__global__ __launch_bounds__(256) void k_forward_tof(LaunchTable T, TofArgs A) {
    extern __shared__ __align__(16) unsigned char tof_lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    // per wave: the queue, then the traversal stack
    unsigned char *base = tof_lds + size_t(wave) * (sizeof(TofQueue) + sizeof(uint32_t) * kWideStack);
    TofQueue &Q = *reinterpret_cast<TofQueue *>(base);
    uint32_t *stack = reinterpret_cast<uint32_t *>(base + sizeof(TofQueue));
    if (T.work_counter) {
        for (int64_t packet = next_packet(T.work_counter, lane); packet < T.n_packets;
             packet = next_packet(T.work_counter, lane))
            packet_forward_tof<kBins>(T, A, packet, lane, stack, Q);
        return;
    }
    const int64_t packet = logical_block(T.xcd_remap) * T.waves_per_group + wave;
    packet_forward_tof<kBins>(T, A, packet, lane, stack, Q);
}

// Gradient sums of one (ray, Gaussian) pair with the ray's bin weights wi[64 b].
template <int kBins>
__device__ inline void pair_grad_tof(const GaussRec &G, float rho, const TofRayF &r, const float *wi,
                                     const TofBins &tb, float k2, float c[10]) {
    double o[3], d[3], dd[6];
    for (int k = 0; k < 3; ++k) {
        o[k] = r.o[k];
        d[k] = r.d[k];
    }
    ray_dd(d, dd);
    PairCore pc;
    pair_core(G.mu, G.P, o, d, dd, pc);
    float D, rr;
    pair_D(pc, D, rr);
    if (!(D <= k2)) return;
    double ra = double(rr * rr);
    ra = fma(ra, fma(-pc.A, ra, 1.0), ra);
    const double t = pc.B * ra;  // -t*
    const float p0 = float(fma(-t, d[0], pc.dl[0]));
    const float p1 = float(fma(-t, d[1], pc.dl[1]));
    const float p2 = float(fma(-t, d[2], pc.dl[2]));
    const float E = kSqrt2Pi * rr * gauss_exp(D);  // unit-density line integral
    const float Tv = E * rho;
    const float iA = float(ra);
    float W, alpha = 0.0f, beta;
    if (tb.nb == 0) {
        W = wi[0];
        beta = W * Tv * iA;
    } else {
        const double s2d = double(tb.sigma2) + ra;
        const float s2 = float(s2d);
        const float is2 = __builtin_amdgcn_rcpf(s2);  // (1 ulp; the moments need no more)
        const float kg = tb.kw * __builtin_amdgcn_rsqf(s2);
        const double u0 = (double(r.c) - tb.half) + t;
        BinChain ch(-0.5 * kLog2eD * rcp_newton(s2d), u0, tb.wd);
        const float uf = float(u0), wf = float(tb.wd);
        float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
        // bin b: weight v_b times g_b, and its moments in tau_b - t*
        auto add = [&](int b, float g) {
            const float u = fmaf(float(b), wf, uf);
            const float vg = wi[64 * b] * g;
            S0 += vg;
            S1 = fmaf(vg, u, S1);
            S2 = fmaf(vg * u, u, S2);
        };
        if (ch.fast()) {
            double g, rb, K;
            ch.start(g, rb, K);
            g *= double(kg);  // the bins' common factor w / sqrt(2 pi s^2), of order one
            // four bins at a time, their weights read together (the rows are
            // padded with zeros to a multiple of four)
            for (int b0 = 0; b0 < tb.nb; b0 += 4) {
                float wv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) wv[k] = wi[64 * (b0 + k)];
                const float ub = fmaf(float(b0), wf, uf);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (b0 + k >= tb.nb) break;
                    const float u = fmaf(float(k), wf, ub);
                    const float vg = wv[k] * float(g);
                    const float vu = vg * u;
                    S0 += vg;
                    S1 += vu;
                    S2 = fmaf(vu, u, S2);
                    BinChain::step(g, rb, K, S0);
                }
            }
        } else {
#pragma unroll
            for (int b = 0; b < kBins; ++b) {
                if (b >= tb.nb) break;
                add(b, kg * ch.next(S0));
            }
        }
        W = S0;
        const float Wt = S1 * is2;
        const float Ws = 0.5f * is2 * (S2 * is2 - S0);
        alpha = Tv * Wt * iA;
        beta = W * Tv * iA + 2.0f * Tv * Ws * iA * iA;
    }
    const float wT = W * Tv;
    const float f0 = r.d[0], f1 = r.d[1], f2 = r.d[2];
    const float q0 = fmaf(wT, p0, alpha * f0), q1 = fmaf(wT, p1, alpha * f1), q2 = fmaf(wT, p2, alpha * f2);
    const float v0 = fmaf(alpha, p0, beta * f0), v1 = fmaf(alpha, p1, beta * f1), v2 = fmaf(alpha, p2, beta * f2);
    c[0] = fmaf(W, E, c[0]);
    c[1] += q0;
    c[2] += q1;
    c[3] += q2;
    c[4] = fmaf(q0, p0, fmaf(v0, f0, c[4]));
    c[5] = fmaf(q1, p1, fmaf(v1, f1, c[5]));
    c[6] = fmaf(q2, p2, fmaf(v2, f2, c[6]));
    c[7] = fmaf(q0, p1, fmaf(v0, f1, c[7]));
    c[8] = fmaf(q0, p2, fmaf(v0, f2, c[8]));
    c[9] = fmaf(q1, p2, fmaf(v1, f2, c[9]));
}

// Backward replay: a lane stores its sums for an entry into the window's LDS
// slot when it moves on, the sums of the entry its range ends in go in by
// close_window; at the end lane q adds entry q's ten sums to the global
// accumulators (one set per (packet, Gaussian)).
template <int kBins>
__device__ inline void replay_backward(const SceneView &S, const TofWave<TofWinB> &L, const TofPending &pe,
                                       const TofRayF &mine, int lane, float k2, const TofBins &tb, float *acc) {
    TofWinB &W = *L.win;
    if (lane < pe.n)
        for (int k = 0; k < 10; ++k) W.res[k][lane] = 0.0f;
    const TofShare sh = stage_window(S, W, pe, lane);
    int e = sh.e;
    uint64_t m = sh.m;
    GaussRec G = W.rec[e];
    float rho = G.rho_c * (1.0f / kSqrt2Pi);
    float c[10];
    for (int k = 0; k < 10; ++k) c[k] = 0.0f;
    for (int it = 0; it < sh.s; ++it) {
        const bool act = it < sh.left;
        if (act && m == 0) {
            // this lane holds the entry's last pair, so no other lane leaves
            // it inside the loop and its slot is still zero
            for (int k = 0; k < 10; ++k) {
                W.res[k][e] = c[k];
                c[k] = 0.0f;
            }
            e = min(e + 1, pe.n - 1);
            m = W.m[e];
            G = W.rec[e];
            rho = G.rho_c * (1.0f / kSqrt2Pi);
        }
        const int i = act ? __builtin_ctzll(m) : lane;
        const TofRayF r = gather_tof_ray(mine, i);
        if (act) {
            m &= m - 1;
            pair_grad_tof<kBins>(G, rho, r, L.bins + i, tb, k2, c);
        }
    }
    close_window<kTofWin>(W.part, W.res, c, sh.left > 0 ? e : -1, lane);
    if (lane < pe.n)
        for (int k = 0; k < 10; ++k) atomicAdd(&acc[k * S.n + pe.g], W.res[k][lane]);
    __builtin_amdgcn_wave_barrier();
}

template <int kBins>
__device__ inline void packet_backward_tof(const LaunchTable &T, const TofArgs &A, int64_t packet, int lane,
                                           const TofWave<TofWinB> &L) {
    PacketRef P;
    if (!locate_packet(T, packet, lane, P)) return;
    const Segment &sg = T.segs[P.seg];
    const SceneView &S = T.scenes[sg.scene];
    Ray R;
    load_ray(sg.ro, sg.rd, sg.stride, P.ray, R);
    Beam B;
    build_beam(R, B);
    const float k2 = S.kappa2;
    const TofBins tb = tof_bins(A);
    const int nw = tb.nb > 0 ? tb.nb : 1;
    // the ray's attenuated bin weights at its lane's slot (zero rows pad them
    // to a multiple of four)
    bool live = false;
    const float a = P.active ? ray_atten(A, P.ray) : 0.0f;
#pragma unroll
    for (int b = 0; b < tof_rows(kBins); ++b) {
        if (b < tof_rows(nw)) {
            const float v = P.active && b < nw ? a * A.grad_out[int64_t(b) * A.n_rays + P.out] : 0.0f;
            L.bins[64 * b + lane] = v;
            live |= v != 0.0f;
        }
    }
    if (ballot(live) == 0) return;
    TofRayF mine;
    for (int k = 0; k < 3; ++k) {
        mine.o[k] = R.o[k];
        mine.d[k] = R.d[k];
    }
    mine.c = ray_center(A, P.ray);
    float *acc = A.acc;
    TofPending pe{0, 0u, 0ull};
    traverse_any(T.traversal, S, R, B, live, lane, L.stack, [&](int l) {
        int64_t start;
        uint64_t mask = leaf_candidates(S, B, l, lane, start);
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
            const uint64_t h0 = ballot(live && D <= k2);
            if (h0) pe.put(lane, start + j0, h0);
            if (two) {
                pair_core(G1.mu, G1.P, R.o64, R.d64, R.dd, c);
                pair_D(c, D, r);
                const uint64_t h1 = ballot(live && D <= k2);
                if (h1) pe.put(lane, start + j1, h1);
            }
            if (pe.n > kTofWin - 2) {
                replay_backward<kBins>(S, L, pe, mine, lane, k2, tb, acc);
                pe.n = 0;
            }
        }
    });
    if (pe.n > 0) replay_backward<kBins>(S, L, pe, mine, lane, k2, tb, acc);
}

template <int kBins>
__global__ __launch_bounds__(256) void k_backward_tof(LaunchTable T, TofArgs A) {
    extern __shared__ __align__(16) unsigned char tof_lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const TofWave<TofWinB> L = tof_wave<TofWinB>(tof_lds, wave, tof_rows(A.n_bins > 0 ? A.n_bins : 1));
    if (T.work_counter) {
        for (int64_t packet = next_packet(T.work_counter, lane); packet < T.n_packets;
             packet = next_packet(T.work_counter, lane))
            packet_backward_tof<kBins>(T, A, packet, lane, L);
        return;
    }
    const int64_t packet = logical_block(T.xcd_remap) * T.waves_per_group + wave;
    packet_backward_tof<kBins>(T, A, packet, lane, L);
}

// TOF centre of each ray: the parameter where it passes closest to the z axis
// in the transaxial plane, -(o_xy . d_xy) / |d_xy|^2 (0 for axial rays). For a
// PET line it is the midpoint of its two end points on the detector cylinder.
__global__ void k_tof_centers(const float *__restrict__ ro, const float *__restrict__ rd, int64_t n,
                              float *__restrict__ center) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ox = ro[i], oy = ro[n + i], dx = rd[i], dy = rd[n + i];
    const double a = dx * dx + dy * dy;
    center[i] = a > 0.0 ? float(-(ox * dx + oy * dy) / a) : 0.0f;
}

// Per-measurement loss weights dL/dI and the loss (summed in FP64): L2
// L = (I - y)^2 / 2, w = I - y; Poisson L = Ib - y log Ib, w = 1 - y / Ib with
// Ib = I + background (per element when bg_arr is given: randoms and scatter
// as expected counts). A bounded grid strides over the elements; each block
// reduces its terms in LDS and adds them with one atomic, so the single loss
// address sees a few thousand atomics, not one per wave.
constexpr int kLossThreads = 256;
__global__ __launch_bounds__(kLossThreads) void k_loss_weights(int32_t kind, const float *__restrict__ I,
                                                               const float *__restrict__ y,
                                                               const float *__restrict__ bg_arr, float bg,
                                                               int64_t count, float *__restrict__ w,
                                                               double *__restrict__ loss) {
    __shared__ double part[kLossThreads / 64];
    double term = 0.0;
    const int64_t stride = int64_t(gridDim.x) * kLossThreads;
    for (int64_t i = int64_t(blockIdx.x) * kLossThreads + threadIdx.x; i < count; i += stride) {
        if (kind == GR_LOSS_L2) {
            const float e = I[i] - y[i];
            term += 0.5 * double(e) * double(e);
            w[i] = e;
        } else {
            const double Ib = double(I[i]) + double(bg_arr ? bg_arr[i] : bg);
            const double yi = y[i];
            term += Ib - yi * log(Ib);
            w[i] = float(1.0 - yi / Ib);
        }
    }
    if (!loss) return;
    for (int off = 32; off >= 1; off >>= 1) term += __shfl_xor(term, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = term;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kLossThreads / 64; ++k) t += part[k];
        atomicAdd(loss, t);
    }
}

template <int kBins>
hipError_t launch_forward(LaunchTable &T, const TofArgs &A, const LaunchShape &shape, hipStream_t st) {
    const unsigned groups = launch_groups(T, shape);
    const size_t lds = (sizeof(TofQueue) + sizeof(uint32_t) * kWideStack) * size_t(shape.waves);
    k_forward_tof<kBins><<<dim3(groups), dim3(64 * shape.waves), lds, st>>>(T, A);
    return hipGetLastError();
}

template <int kBins>
hipError_t launch_backward(LaunchTable &T, const TofArgs &A, const LaunchShape &shape, hipStream_t st) {
    const unsigned groups = launch_groups(T, shape);
    const size_t lds = tof_wave_bytes<TofWinB>(tof_rows(A.n_bins > 0 ? A.n_bins : 1)) * size_t(shape.waves);
    k_backward_tof<kBins><<<dim3(groups), dim3(64 * shape.waves), lds, st>>>(T, A);
    return hipGetLastError();
}

}  // namespace

int tof_bins_class(int n_bins) { return n_bins <= 1 ? 1 : n_bins <= 8 ? 8 : n_bins <= 16 ? 16 : 32; }

hipError_t enqueue_forward_tof(LaunchTable &T, const TofArgs &A, const LaunchShape &shape, hipStream_t st) {
    finish_table(T, shape);
    if (T.n_packets == 0) return hipSuccess;
    if (shape.work_counter) enqueue_zero_u32(shape.work_counter, st);
    switch (tof_bins_class(A.n_bins)) {
        case 1: return launch_forward<1>(T, A, shape, st);
        case 8: return launch_forward<8>(T, A, shape, st);
        case 16: return launch_forward<16>(T, A, shape, st);
        default: return launch_forward<32>(T, A, shape, st);
    }
}

hipError_t enqueue_backward_tof(LaunchTable &T, const TofArgs &A, const gr_scene &sc, const uint32_t *order,
                                float *gmean, float *gscale, float *gquat, float *gdens, const LaunchShape &shape,
                                hipStream_t st) {
    finish_table(T, shape);
    enqueue_zero_f32(A.acc, 10 * sc.n, st);
    if (T.n_packets > 0) {
        if (shape.work_counter) enqueue_zero_u32(shape.work_counter, st);
        hipError_t e;
        switch (tof_bins_class(A.n_bins)) {
            case 1: e = launch_backward<1>(T, A, shape, st); break;
            case 8: e = launch_backward<8>(T, A, shape, st); break;
            case 16: e = launch_backward<16>(T, A, shape, st); break;
            default: e = launch_backward<32>(T, A, shape, st); break;
        }
        if (e != hipSuccess) return e;
    }
    enqueue_epilogue(sc, order, A.acc, gmean, gscale, gquat, gdens, st);
    return hipGetLastError();
}

hipError_t enqueue_tof_centers(const float *ro, const float *rd, int64_t n, float *center, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_tof_centers<<<unsigned((n + 255) / 256), 256, 0, st>>>(ro, rd, n, center);
    return hipGetLastError();
}

hipError_t enqueue_loss_weights(int32_t kind, const float *proj, const float *target, const float *bg_arr,
                                float bg, int64_t count, float *weight, double *loss, hipStream_t st) {
    if (count == 0) return hipSuccess;
    // enough blocks to fill the chip (256 CUs x 8), never more than the work
    const int64_t blocks = std::min<int64_t>((count + kLossThreads - 1) / kLossThreads, 2048);
    k_loss_weights<<<unsigned(blocks), kLossThreads, 0, st>>>(kind, proj, target, bg_arr, bg, count, weight, loss);
    return hipGetLastError();
}

}  // namespace gr
