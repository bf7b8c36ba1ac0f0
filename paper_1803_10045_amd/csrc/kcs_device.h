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
__device__ __forceinline__ void load_record(const float* __restrict__ p, float (&v)[M]) {
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
__device__ __forceinline__ void store_record(float* __restrict__ p, const float (&v)[M]) {
#pragma unroll
    for (int k = 0; k < M / 4; ++k)
        reinterpret_cast<float4*>(p)[k] = make_float4(v[4 * k + 0], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}

// Constants of projection angle a: t_a = ang0 + a pi / n_ang, cos and sin computed in FP64 and
// snapped exactly at multiples of pi/2, then rounded to FP32.
__device__ __forceinline__ AngleRec make_angle(int a, int n_ang, double ang0, float h) {
    const double t = ang0 + (double)a * 3.141592653589793 / (double)n_ang;
    double s, c;
    sincos(t, &s, &c);
    if (fabs(c) < 1e-12) {
        c = 0.0;
        s = s > 0.0 ? 1.0 : -1.0;
    }
    if (fabs(s) < 1e-12) {
        s = 0.0;
        c = c > 0.0 ? 1.0 : -1.0;
    }
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

// Chord of a ray through a pixel square: the exact intersection length as a function of the
// signed distance t between the ray and the pixel centre, measured along the detector.
__device__ __forceinline__ float pixel_chord(const AngleRec& A, float t) {
    if (A.axis == 0) {
        const float f = fminf(fmaxf((A.w1 - fabsf(t)) * A.inv_dw, 0.0f), 1.0f);
        return A.m * f;
    }
    // axis-aligned: the pixel is hit iff the ray lies in its half-open extent
    const float cs = A.axis == 1 ? A.c : A.s;
    const float w0 = A.w1;
    const bool in = cs > 0.0f ? (t >= -w0 && t < w0) : (t > -w0 && t <= w0);
    return in ? A.m : 0.0f;
}

}  // namespace kcs
