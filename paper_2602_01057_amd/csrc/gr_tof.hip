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
// rays); kBins accumulators per lane (FP64), bins guarded by n_bins. The
// backward is Gaussian-major with the packet's rays, centres and bin weights
// staged in LDS.
#include <algorithm>

#include "gr_trace.h"

namespace gr {

namespace {

constexpr double kLog2eD = 1.4426950408889634074;

// A ray of a TOF backward packet (FP32 inputs widened, exact).
struct TofRay {
    double o[3];
    double d[3];
};

// Rays of a TOF backward packet, staged in LDS.
template <int kBins>
struct TofRays {
    TofRay rays[64];
    float center[64];
    float w[kBins][64];
};

template <int kBins>
struct TofLds {
    TofRays<kBins> r;
    int32_t cand[128];
    uint32_t stack[kWideStack];
};

__device__ inline float ray_center(const TofArgs &A, int64_t ray) { return A.center ? A.center[ray] : 0.0f; }
__device__ inline float ray_atten(const TofArgs &A, int64_t ray) { return A.atten ? A.atten[ray] : 1.0f; }

// One packet of the TOF forward.
template <int kBins>
__device__ inline void packet_forward_tof(const LaunchTable &T, const TofArgs &A, int64_t packet, int lane,
                                          uint32_t *stack) {
    PacketRef P;
    if (!locate_packet(T, packet, lane, P)) return;
    const Segment &sg = T.segs[P.seg];
    const SceneView S = T.scenes[sg.scene];
    Ray R;
    load_ray(sg.ro, sg.rd, sg.stride, P.ray, R);
    Beam B;
    build_beam(R, B);
    const float k2 = S.kappa2;
    const int nb = A.n_bins;
    const bool tof = nb > 0;
    // bin b's centre minus t* is (c - b0 w) + b w - t*, b0 = (nb - 1)/2
    const double c0 = double(ray_center(A, P.ray)) - 0.5 * double(nb - 1) * double(A.width);
    const double wd = A.width;
    const float kw = A.width * 0.39894228040143268f;  // w / sqrt(2 pi)
    double acc[kBins];
#pragma unroll
    for (int b = 0; b < kBins; ++b) acc[b] = 0.0;
    traverse_any(T.traversal, S, R, B, P.active, lane, stack, [&](int l) {
        int64_t start;
        uint64_t mask = leaf_candidates(S, B, l, lane, start);
        while (mask) {
            const int j = __builtin_ctzll(mask);
            mask &= mask - 1;
            const GaussRec G = sload(S.rec, start + j);
            PairCore c;
            float D, r;
            pair_core(G.mu, G.P, R.o64, R.d64, R.dd, c);
            pair_D(c, D, r);
            if (!(D <= k2)) continue;
            const float Tv = G.rho_c * r * gauss_exp(D);
            if (!tof) {
                acc[0] += double(Tv);
                continue;
            }
            // 1/A from the FP32 r^2 and one Newton step, t* = -B/A in FP64
            double ra = double(r * r);
            ra = fma(ra, fma(-c.A, ra, 1.0), ra);
            const double u0 = c0 + c.B * ra;  // tau_0 - t*
            const double s2d = double(A.sigma2) + ra;
            const float s2 = float(s2d);
            // the exponent in FP64, rounded once: deep in the kernel's tail
            // (|exponent| ~ 100) an FP32 product chain would cost ~1e-5
            const double qd = -0.5 * kLog2eD / s2d;
            const float Tg = Tv * kw * __builtin_amdgcn_rsqf(s2);
#pragma unroll
            for (int b = 0; b < kBins; ++b) {
                if (b < nb) {
                    const double u = fma(double(b), wd, u0);
                    acc[b] += double(Tg * __builtin_amdgcn_exp2f(float(qd * u * u)));
                }
            }
        }
    });
    if (P.active) {
        const float a = ray_atten(A, P.ray);
        const int nout = tof ? nb : 1;
#pragma unroll
        for (int b = 0; b < kBins; ++b)
            if (b < nout) A.out[int64_t(b) * A.n_rays + P.out] = float(double(a) * acc[b]);
    }
}

template <int kBins>
__global__ __launch_bounds__(256) void k_forward_tof(LaunchTable T, TofArgs A) {
    extern __shared__ uint32_t tof_stack[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    uint32_t *stack = tof_stack + wave * kWideStack;
    if (T.work_counter) {
        for (int64_t packet = next_packet(T.work_counter, lane); packet < T.n_packets;
             packet = next_packet(T.work_counter, lane))
            packet_forward_tof<kBins>(T, A, packet, lane, stack);
        return;
    }
    const int64_t packet = logical_block(T.xcd_remap) * T.waves_per_group + wave;
    packet_forward_tof<kBins>(T, A, packet, lane, stack);
}

// Gradient sums of one (ray, Gaussian) pair with the ray's bins.
template <int kBins>
__device__ inline void pair_grad_tof(const GaussRec &G, float rho, const TofRays<kBins> &Rs, int i, int nb,
                                     float sigma2, float width, float k2, float c[10], bool &any) {
    const TofRay &Rr = Rs.rays[i];
    double dd[6];
    ray_dd(Rr.d, dd);
    PairCore pc;
    pair_core(G.mu, G.P, Rr.o, Rr.d, dd, pc);
    float D, r;
    pair_D(pc, D, r);
    if (!(D <= k2)) return;
    any = true;
    double ra = double(r * r);
    ra = fma(ra, fma(-pc.A, ra, 1.0), ra);
    const double t = pc.B * ra;  // -t*
    const float p0 = float(fma(-t, Rr.d[0], pc.dl[0]));
    const float p1 = float(fma(-t, Rr.d[1], pc.dl[1]));
    const float p2 = float(fma(-t, Rr.d[2], pc.dl[2]));
    const float E = kSqrt2Pi * r * gauss_exp(D);  // unit-density line integral
    const float Tv = E * rho;
    const float iA = float(ra);
    float W, alpha = 0.0f, beta;
    if (nb == 0) {
        W = Rs.w[0][i];
        beta = W * Tv * iA;
    } else {
        const double s2d = double(sigma2) + ra;
        const float s2 = float(s2d);
        const float is2 = 1.0f / s2;
        const double qd = -0.5 * kLog2eD / s2d;
        const float kg = width * 0.39894228040143268f * __builtin_amdgcn_rsqf(s2);
        const double u0 = double(Rs.center[i]) - 0.5 * double(nb - 1) * double(width) + t;
        float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
#pragma unroll
        for (int b = 0; b < kBins; ++b) {
            if (b < nb) {
                const double ud = fma(double(b), double(width), u0);
                const float u = float(ud);
                const float vg = Rs.w[b][i] * kg * __builtin_amdgcn_exp2f(float(qd * ud * ud));
                S0 += vg;
                S1 = fmaf(vg, u, S1);
                S2 = fmaf(vg * u, u, S2);
            }
        }
        W = S0;
        const float Wt = S1 * is2;
        const float Ws = 0.5f * is2 * (S2 * is2 - S0);
        alpha = Tv * Wt * iA;
        beta = W * Tv * iA + 2.0f * Tv * Ws * iA * iA;
    }
    const float wT = W * Tv;
    const float f0 = float(Rr.d[0]), f1 = float(Rr.d[1]), f2 = float(Rr.d[2]);
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

// One batch of up to 64 candidates (lane j owns cand[j]) against the live rays.
template <int kBins>
__device__ inline void backward_batch_tof(const SceneView &S, const TofLds<kBins> &L, int cnt, uint64_t live,
                                          int lane, int nb, float sigma2, float width, float k2, float *acc) {
    const bool own = lane < cnt;
    const int64_t g = own ? L.cand[lane] : L.cand[0];
    const GaussRec G = S.rec[g];
    const float rho = G.rho_c * (1.0f / kSqrt2Pi);
    float c[10];
    for (int k = 0; k < 10; ++k) c[k] = 0.0f;
    bool any = false;
    for (uint64_t lm = live; lm; lm &= lm - 1)
        pair_grad_tof<kBins>(G, rho, L.r, __builtin_ctzll(lm), nb, sigma2, width, k2, c, any);
    if (own && any)
        for (int k = 0; k < 10; ++k) atomicAdd(&acc[k * S.n + g], c[k]);
}

template <int kBins>
__device__ inline void packet_backward_tof(const LaunchTable &T, const TofArgs &A, int64_t packet, int lane,
                                           TofLds<kBins> *L) {
    PacketRef P;
    if (!locate_packet(T, packet, lane, P)) return;
    const Segment &sg = T.segs[P.seg];
    const SceneView S = T.scenes[sg.scene];
    Ray R;
    load_ray(sg.ro, sg.rd, sg.stride, P.ray, R);
    Beam B;
    build_beam(R, B);
    const float k2 = S.kappa2;
    const int nb = A.n_bins;
    const int nw = nb > 0 ? nb : 1;
    // stage the ray, its centre and its attenuated bin weights at its lane's slot
    bool live = false;
    if (P.active) {
        const float a = ray_atten(A, P.ray);
#pragma unroll
        for (int b = 0; b < kBins; ++b) {
            if (b < nw) {
                const float v = a * A.grad_out[int64_t(b) * A.n_rays + P.out];
                L->r.w[b][lane] = v;
                live |= v != 0.0f;
            }
        }
        TofRay &rr = L->r.rays[lane];
        for (int k = 0; k < 3; ++k) {
            rr.o[k] = R.o64[k];
            rr.d[k] = R.d64[k];
        }
        L->r.center[lane] = ray_center(A, P.ray);
    }
    const uint64_t live_mask = ballot(live);
    if (live_mask == 0) return;
    __builtin_amdgcn_wave_barrier();
    float *acc = A.acc;
    int count = 0;
    traverse_any(T.traversal, S, R, B, live, lane, L->stack, [&](int l) {
        int64_t start;
        const uint64_t mask = leaf_candidates(S, B, l, lane, start);
        if (!mask) return;
        if ((mask >> lane) & 1ull) {
            const int pos = count + __builtin_popcountll(mask & ((1ull << lane) - 1ull));
            L->cand[pos] = int32_t(start + lane);
        }
        count += __builtin_popcountll(mask);
        __builtin_amdgcn_wave_barrier();
        if (count >= 64) {
            backward_batch_tof<kBins>(S, *L, 64, live_mask, lane, nb, A.sigma2, A.width, k2, acc);
            const int rest = count - 64;
            int moved = 0;
            if (lane < rest) moved = L->cand[64 + lane];
            __builtin_amdgcn_wave_barrier();
            if (lane < rest) L->cand[lane] = moved;
            __builtin_amdgcn_wave_barrier();
            count = rest;
        }
    });
    if (count > 0) backward_batch_tof<kBins>(S, *L, count, live_mask, lane, nb, A.sigma2, A.width, k2, acc);
}

template <int kBins>
__global__ __launch_bounds__(256) void k_backward_tof(LaunchTable T, TofArgs A) {
    extern __shared__ __align__(16) unsigned char tof_lds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    TofLds<kBins> *L = reinterpret_cast<TofLds<kBins> *>(tof_lds) + wave;
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
    const size_t lds = sizeof(uint32_t) * kWideStack * size_t(shape.waves);
    k_forward_tof<kBins><<<dim3(groups), dim3(64 * shape.waves), lds, st>>>(T, A);
    return hipGetLastError();
}

template <int kBins>
hipError_t launch_backward(LaunchTable &T, const TofArgs &A, const LaunchShape &shape, hipStream_t st) {
    const unsigned groups = launch_groups(T, shape);
    const size_t lds = sizeof(TofLds<kBins>) * size_t(shape.waves);
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
