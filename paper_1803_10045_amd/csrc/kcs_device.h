// Device helpers shared by the kernels of libkcs.
#pragma once

#include "kcs_internal.h"

namespace kcs {

// The hardware hands consecutive workgroup ids to the 8 XCDs round-robin.  Remap the linear
// workgroup id so that each XCD walks one contiguous slice of the work list (neighbouring
// tiles of the same planes then share that XCD's L2).  `n_groups` is the launched grid size,
// a multiple of 8; returns the work index for this workgroup.
constexpr int kXcds = 8;

__device__ __forceinline__ uint32_t xcd_work_index(uint32_t bid, uint32_t n_groups) {
    const uint32_t per = n_groups / kXcds;
    return (bid % kXcds) * per + bid / kXcds;
}

__host__ __device__ inline uint32_t xcd_round_up(uint32_t n) { return (n + kXcds - 1) / kXcds * kXcds; }

template <int M>
__host__ __device__ __forceinline__ void load_record(const float* __restrict__ p, float (&v)[M]) {
    static_assert(M % 4 == 0, "frames must be a multiple of 4");
#pragma unroll
    for (int k = 0; k < M / 4; ++k) {
        const float4 q = reinterpret_cast<const float4*>(p)[k];
        v[4 * k + 0] = q.x;
        v[4 * k + 1] = q.y;
        v[4 * k + 2] = q.z;
        v[4 * k + 3] = q.w;
    }
}

template <int M>
__host__ __device__ __forceinline__ void store_record(float* __restrict__ p, const float (&v)[M]) {
#pragma unroll
    for (int k = 0; k < M / 4; ++k)
        reinterpret_cast<float4*>(p)[k] = make_float4(v[4 * k + 0], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}

// cos and sin of projection angle a, t_a = ang0 + a pi / n_ang, in FP64, snapped exactly at
// multiples of pi/2.
__host__ __device__ inline void angle_cos_sin(int a, int n_ang, double ang0, double& c, double& s) {
    const double t = ang0 + (double)a * 3.141592653589793 / (double)n_ang;
    sincos(t, &s, &c);
    if (fabs(c) < 1e-12) {
        c = 0.0;
        s = s > 0.0 ? 1.0 : -1.0;
    }
    if (fabs(s) < 1e-12) {
        s = 0.0;
        c = c > 0.0 ? 1.0 : -1.0;
    }
}

// Constants of a projection angle from its FP64 cos and sin (rounded to FP32).
__host__ __device__ inline AngleRec make_angle_cs(double c, double s, float h) {
    const double ac = fabs(c), as = fabs(s), hd = (double)h;
    AngleRec A;
    A.c = (float)c;
    A.s = (float)s;
    A.inv_c = c != 0.0 ? (float)(1.0 / c) : 0.0f;
    A.inv_s = s != 0.0 ? (float)(1.0 / s) : 0.0f;
    A.m = (float)(hd / fmax(ac, as));
    A.w1 = (float)(0.5 * hd * (ac + as));
    A.axis = s == 0.0 ? 1 : (c == 0.0 ? 2 : 0);
    A.inv_dw = A.axis == 0 ? (float)(1.0 / (hd * fmin(ac, as))) : 0.0f;
    return A;
}

// Constants of projection angle a.
__host__ __device__ inline AngleRec make_angle(int a, int n_ang, double ang0, float h) {
    double s, c;
    angle_cos_sin(a, n_ang, ang0, c, s);
    return make_angle_cs(c, s, h);
}

// 1 / b from the hardware reciprocal (1 ulp) for normal positive b; exact on the host.
__host__ __device__ __forceinline__ float recip(float b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(b);
#else
    return 1.0f / b;
#endif
}

// Chord of a ray through a pixel square: the exact intersection length as a function of the
// signed distance t between the ray and the pixel centre, measured along the detector; for
// oblique angles a trapezoid in t.
__host__ __device__ __forceinline__ float chord_oblique(const AngleRec& A, float t) {
    return A.m * fminf(fmaxf((A.w1 - fabsf(t)) * A.inv_dw, 0.0f), 1.0f);
}

// Axis-aligned angles: the pixel is hit iff the ray lies in its half-open extent.
__host__ __device__ __forceinline__ float chord_axis(const AngleRec& A, float t) {
    const float cs = A.axis == 1 ? A.c : A.s;
    const float w0 = A.w1;
    const bool in = cs > 0.0f ? (t >= -w0 && t < w0) : (t > -w0 && t <= w0);
    return in ? A.m : 0.0f;
}

__host__ __device__ __forceinline__ float pixel_chord(const AngleRec& A, float t) {
    return A.axis == 0 ? chord_oblique(A, t) : chord_axis(A, t);
}

// Incremental Siddon traversal of a ray through an nx x ny box of pixels: calls
// visit(j * row + i * col, len) for every pixel (i, j) the ray crosses, in order, with the exact
// intersection length (mm).  Coordinates are in pixel units relative to the box corner; (Xc, Yc) is a point
// of the ray and the point at parameter lam (pixel units of length) is (Xc - lam s, Yc + lam c).  The
// crossing parameters are re-derived from the grid-line index at each step, so the rounding
// error does not accumulate along the ray.  At most nx + ny + 2 steps.
template <class Visit>
__host__ __device__ __forceinline__ void siddon_traverse_box(const AngleRec& A, float Xc, float Yc, int nx, int ny,
                                                             float h, int row, int col, Visit&& visit) {
    float lin = -3.0e38f, lout = 3.0e38f;
    bool hit = true;
    if (A.s != 0.0f) {
        const float l0 = Xc * A.inv_s, l1 = (Xc - (float)nx) * A.inv_s;
        lin = fmaxf(lin, fminf(l0, l1));
        lout = fminf(lout, fmaxf(l0, l1));
    } else {
        hit = hit && Xc >= 0.0f && Xc < (float)nx;
    }
    if (A.c != 0.0f) {
        const float l0 = -Yc * A.inv_c, l1 = ((float)ny - Yc) * A.inv_c;
        lin = fmaxf(lin, fminf(l0, l1));
        lout = fminf(lout, fmaxf(l0, l1));
    } else {
        hit = hit && Yc >= 0.0f && Yc < (float)ny;
    }
    if (!(hit && lout > lin)) return;
    // first pixel: the one the ray enters, judged by its direction of travel
    int i, j, si = 0, sj = 0;
    if (A.s != 0.0f) {
        const float Xin = Xc - lin * A.s;
        si = A.s < 0.0f ? 1 : -1;
        i = si > 0 ? (int)floorf(Xin) : (int)ceilf(Xin) - 1;
        i = min(max(i, 0), nx - 1);
    } else {
        i = (int)floorf(Xc);
    }
    if (A.c != 0.0f) {
        const float Yin = Yc + lin * A.c;
        sj = A.c > 0.0f ? 1 : -1;
        j = sj > 0 ? (int)floorf(Yin) : (int)ceilf(Yin) - 1;
        j = min(max(j, 0), ny - 1);
    } else {
        j = (int)floorf(Yc);
    }
    const float bx0 = (float)(si > 0 ? i + 1 : i), by0 = (float)(sj > 0 ? j + 1 : j);
    // crossing parameters in mm of path (pixel units times h), re-derived from the number of
    // grid lines crossed; a step updates both axes with selects, so the wave does not branch
    const float lx0 = si ? (Xc - bx0) * (A.inv_s * h) : 3.0e38f;
    const float ly0 = sj ? (by0 - Yc) * (A.inv_c * h) : 3.0e38f;
    const float dlx = si ? fabsf(A.inv_s * h) : 0.0f, dly = sj ? fabsf(A.inv_c * h) : 0.0f;
    float lx = lx0, ly = ly0, lcur = lin * h;
    // The walk ends at the first grid line of the box's far edges, taken from the same formula
    // as the steps: fma(k, d, l0) is monotone in k, so no step can pass that line and (i, j)
    // stays inside the box without a bounds test (in exact arithmetic this is lout).
    const int nlx = si > 0 ? nx - 1 - i : (si < 0 ? i : 0);
    const int nly = sj > 0 ? ny - 1 - j : (sj < 0 ? j : 0);
    const float lend = fminf(lout * h, fminf(fmaf((float)nlx, dlx, lx0), fmaf((float)nly, dly, ly0)));
    float kx = 0.0f, ky = 0.0f;
    // the pixel's offset j * row + i * col is stepped along with (i, j): no multiplies
    int idx = j * row + i * col;
    const int dix = si * col, diy = sj * row;
    const int max_steps = nx + ny + 2;
    // two crossings per loop pass: the loop-back branch and the copies of lnext and of the
    // pixel offset come once per two crossings
#pragma unroll 2
    for (int step = 0; step < max_steps; ++step) {
        const float lnext = fminf(fminf(lx, ly), lend);
        visit(idx, lnext - lcur);
        if (lnext >= lend) break;
        const bool sx = lx <= ly;
        kx += sx ? 1.0f : 0.0f;
        ky += sx ? 0.0f : 1.0f;
        idx += sx ? dix : diy;
        lx = fmaf(kx, dlx, lx0);
        ly = fmaf(ky, dly, ly0);
        lcur = lnext;
    }
}

// Slots reserved per (tile, angle) for the bins whose rays can meet a T x T pixel tile:
// b1 - b0 <= T h sqrt(2) / du + 0.02 for every angle (see box_bins).
__host__ __device__ inline int tile_slots(int T, float h, float du) {
    return (int)floorf((float)T * h * 1.41421357f / du) + 3;
}

// Bins whose rays can meet the pixel box [i0, i0+w) x [j0, j0+hgt) of an nx x ny grid: the
// box's corners projected on the detector, widened by a hundredth of a bin so that rounding can
// only add rays (a ray that misses the box contributes exactly 0).  Producer and consumer of
// per-tile partial sums call this same function, so they agree on the set.
__host__ __device__ __forceinline__ void box_bins(const AngleRec& A, int i0, int j0, int w, int hgt, int nx, int ny,
                                                  float h, float inv_du, int n_bin, int& b0, int& b1) {
    const float xl = ((float)i0 - 0.5f * (float)nx) * h, xr = xl + (float)w * h;
    const float yl = ((float)j0 - 0.5f * (float)ny) * h, yr = yl + (float)hgt * h;
    const float u0 = xl * A.c, u1 = xr * A.c, v0 = yl * A.s, v1 = yr * A.s;
    const float umin = fminf(u0, u1) + fminf(v0, v1), umax = fmaxf(u0, u1) + fmaxf(v0, v1);
    const float bc = 0.5f * (float)(n_bin - 1);
    b0 = max((int)ceilf(fmaf(umin, inv_du, bc) - 0.01f), 0);
    b1 = min((int)floorf(fmaf(umax, inv_du, bc) + 0.01f), n_bin - 1);
}

}  // namespace kcs
