// Ray generation for CT (parallel / cone beam) and cylindrical PET with arc
// correction applied at ray set-up. The paper defines each ray's origin and
// direction from the scanner geometry (Fig. 1) and places PET lines of
// response at their true, non-uniformly spaced chord positions instead of
// resampling the sinogram (Fig. 2, Sec. 3 "Inherent limitations", Sec. 6).
// Computed in FP64, written as FP32 SoA, in the packet order stated in gr.h.
#include <math.h>

#include "gr_internal.h"

namespace gr {

// Inverse of the tiled order inside one view: position -> grid cell (i, j),
// i fastest. Tiles of tu x tv, enumerated tile row by tile row; edge tiles
// are partial.
__device__ inline void untile(int64_t pos, int64_t nu, int64_t nv, int64_t tu, int64_t tv,
                              int64_t &i, int64_t &j) {
    const int64_t tj = pos / (tv * nu);
    const int64_t rem = pos - tj * tv * nu;
    const int64_t ht = min(tv, nv - tj * tv);
    const int64_t ti = rem / (tu * ht);
    const int64_t rem2 = rem - ti * tu * ht;
    const int64_t wt = min(tu, nu - ti * tu);
    i = ti * tu + rem2 % wt;
    j = tj * tv + rem2 / wt;
}

// Inverse of the view-blocked tiled order: views go in blocks of kv (the last
// block may be shorter, V views); inside a block the (i, j) grid is tiled as
// in untile, and each tile holds its cells for every view of the block, view
// by view (row-major inside the tile). A shorter last block whose V divides kv
// takes tiles kv / V times taller, so that its tiles hold as many rays as the
// others. kv = 1 is the per-view order.
__device__ inline void untile_views(int64_t idx, int64_t n_views, int64_t nu, int64_t nv, int64_t tu, int64_t tv0,
                                    int64_t kv, int64_t &v, int64_t &i, int64_t &j) {
    const int64_t per = nu * nv;
    const int64_t b = idx / (kv * per);
    const int64_t V = min(kv, n_views - b * kv);
    const int64_t tv = V < kv && kv % V == 0 ? tv0 * (kv / V) : tv0;
    const int64_t pos = idx - b * kv * per;
    const int64_t tj = pos / (V * tv * nu);
    const int64_t rem = pos - tj * V * tv * nu;
    const int64_t ht = min(tv, nv - tj * tv);
    const int64_t ti = rem / (V * tu * ht);
    const int64_t rem2 = rem - ti * V * tu * ht;
    const int64_t wt = min(tu, nu - ti * tu);
    const int64_t k = rem2 / (wt * ht);
    const int64_t rem3 = rem2 - k * wt * ht;
    v = b * kv + k;
    i = ti * tu + rem3 % wt;
    j = tj * tv + rem3 / wt;
}

__device__ inline void store_ray(float *ro, float *rd, int64_t n, int64_t idx, const double o[3],
                                 const double d[3]) {
    for (int k = 0; k < 3; ++k) {
        ro[k * n + idx] = float(o[k]);
        rd[k * n + idx] = float(d[k]);
    }
}

// o = foot of the perpendicular from the isocentre onto the line through p
// with unit direction d.
__device__ inline void foot(const double p[3], const double d[3], double o[3]) {
    const double t = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
    for (int k = 0; k < 3; ++k) o[k] = p[k] - t * d[k];
}

__global__ __launch_bounds__(256) void k_rays_ct(gr_ct_geom g, int64_t n, float *__restrict__ ro,
                                                 float *__restrict__ rd) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int64_t per = int64_t(g.nu) * g.nv;
    const int64_t v = idx / per;
    int64_t i, j;
    untile(idx - v * per, g.nu, g.nv, g.tile_u, g.tile_v, i, j);
    const double th = g.angle0 + double(v) * (g.angle_range / double(g.n_views));
    double sn, cs;
    sincos(th, &sn, &cs);
    const double es[3] = {cs, sn, 0.0}, eu[3] = {-sn, cs, 0.0};
    const double u = (double(i) - (g.nu - 1) / 2.0) * g.pitch_u + g.offset_u;
    const double w = (double(j) - (g.nv - 1) / 2.0) * g.pitch_v + g.offset_v;
    double o[3], d[3];
    if (g.cone == 0) {
        for (int k = 0; k < 3; ++k) d[k] = -es[k];
        o[0] = u * eu[0];
        o[1] = u * eu[1];
        o[2] = w;
    } else {
        const double S[3] = {g.dso * es[0], g.dso * es[1], 0.0};
        const double P[3] = {-(g.dsd - g.dso) * es[0] + u * eu[0], -(g.dsd - g.dso) * es[1] + u * eu[1], w};
        double len = 0.0;
        for (int k = 0; k < 3; ++k) {
            d[k] = P[k] - S[k];
            len += d[k] * d[k];
        }
        len = sqrt(len);
        for (int k = 0; k < 3; ++k) d[k] /= len;
        foot(S, d, o);
    }
    store_ray(ro, rd, n, idx, o, d);
}

// Default plane list: ring difference 0, +1, -1, +2, -2, ... , each group in
// increasing r1.
__device__ inline void default_plane(int64_t p, int n_rings, int max_diff, int &r1, int &r2) {
    if (p < n_rings) {
        r1 = r2 = int(p);
        return;
    }
    p -= n_rings;
    for (int a = 1; a <= max_diff && a < n_rings; ++a) {
        const int cnt = n_rings - a;
        if (p < cnt) {
            r1 = int(p);
            r2 = r1 + a;
            return;
        }
        p -= cnt;
        if (p < cnt) {
            r1 = int(p) + a;
            r2 = r1 - a;
            return;
        }
        p -= cnt;
    }
    r1 = r2 = 0;
}

__global__ __launch_bounds__(256) void k_rays_pet(gr_pet_geom g, int64_t n_planes, int64_t n,
                                                  float *__restrict__ ro, float *__restrict__ rd) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    int64_t v, kk, p;
    untile_views(idx, g.n_views, g.n_radial, n_planes, g.tile_radial, g.tile_axial, g.tile_views > 1 ? g.tile_views : 1,
                 v, kk, p);
    int r1, r2;
    if (g.planes) {
        r1 = g.planes[2 * p];
        r2 = g.planes[2 * p + 1];
    } else {
        default_plane(p, g.n_rings, g.max_ring_diff, r1, r2);
    }
    const int64_t k = kk - g.n_radial / 2;
    const double N = double(g.n_crystals), Rr = g.ring_radius;
    const double psi = M_PI * double(v) / double(g.n_views) + double(k & 1) * (M_PI / N);
    const double gam = M_PI / 2.0 - M_PI * double(k) / N;
    const double z1 = (double(r1) - (g.n_rings - 1) / 2.0) * g.ring_pitch;
    const double z2 = (double(r2) - (g.n_rings - 1) / 2.0) * g.ring_pitch;
    double sa, ca, sb, cb;
    sincos(psi + gam, &sa, &ca);
    sincos(psi - gam, &sb, &cb);
    double A[3] = {Rr * ca, Rr * sa, z1};
    double Bp[3] = {Rr * cb, Rr * sb, z2};
    if (g.arc_correct == 0) {
        const double shift = double(k) * (M_PI * Rr / N) - Rr * sin(M_PI * double(k) / N);
        double sp, cp;
        sincos(psi, &sp, &cp);
        A[0] += shift * cp;
        A[1] += shift * sp;
        Bp[0] += shift * cp;
        Bp[1] += shift * sp;
    }
    double d[3], len = 0.0;
    for (int c = 0; c < 3; ++c) {
        d[c] = Bp[c] - A[c];
        len += d[c] * d[c];
    }
    len = sqrt(len);
    for (int c = 0; c < 3; ++c) d[c] /= len;
    double o[3];
    foot(A, d, o);
    store_ray(ro, rd, n, idx, o, d);
}

int64_t pet_default_plane_count(int n_rings, int max_diff) {
    int64_t c = n_rings;
    for (int a = 1; a <= max_diff && a < n_rings; ++a) c += 2 * int64_t(n_rings - a);
    return c;
}

hipError_t enqueue_rays_ct(const gr_ct_geom &g, int64_t n, float *ro, float *rd, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_rays_ct<<<unsigned((n + 255) / 256), 256, 0, st>>>(g, n, ro, rd);
    return hipGetLastError();
}

hipError_t enqueue_rays_pet(const gr_pet_geom &g, int64_t n_planes, int64_t n, float *ro, float *rd,
                            hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_rays_pet<<<unsigned((n + 255) / 256), 256, 0, st>>>(g, n_planes, n, ro, rd);
    return hipGetLastError();
}

}  // namespace gr
