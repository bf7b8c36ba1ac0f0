// Internal declarations shared by the host side and the kernels of libkcs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "kcs.h"

namespace kcs {

constexpr int kMaxFrames = 32;
constexpr int kMaxBoundaries = 2 * kMaxFrames;  // frame starts and ends
constexpr int kRates = 3;                       // distinct exponents of the input function
constexpr int kTaylor = 12;                     // terms of the near-singular series
constexpr int kTaylorCoef = kTaylor + 3;        // c_1 .. c_{kTaylor+3}
// The series replaces the divided differences where |(l_i + a) t| < kTaylorR0 + kTaylorR1 |l_i t|:
// there the quotient form loses about (3 + |l_i t|) / |(l_i + a) t| digits per order.
constexpr float kTaylorR0 = 0.5f;
constexpr float kTaylorR1 = 0.25f;

// Per-angle constants of the parallel-beam geometry (FP32 copies of FP64 host values).
struct AngleRec {
    float c, s;        // cos, sin of the ray normal, exact 0/+-1 at multiples of pi/2
    float inv_c, inv_s;  // 1/c, 1/s (0 where c or s is 0)
    float m;           // longest chord of a pixel: h / max(|c|, |s|)
    float w1;          // half-width of the pixel's footprint on the detector: h (|c| + |s|) / 2
    float inv_dw;      // 1 / (w1 - w0) with w0 = h | |c| - |s| | / 2; 0 when axis-aligned
    int32_t axis;      // 0 general, 1 if s == 0, 2 if c == 0
};

// Frame schedule and the voxel-independent integrals of the input function.
struct FrameTab {
    int32_t M;
    int32_t contiguous;  // 1 if t0[m+1] == t1[m] for all m
    float E[kMaxFrames];       // c * dt_m
    float r[kMaxFrames];       // background per bin
    float inv_dt[kMaxFrames];  // 1 / dt_m
    float blood[kMaxFrames];   // vb * int_frame Cp
    float dP2[kMaxFrames];     // int_frame P1 (= P2(t1) - P2(t0))
    float cp_int[kMaxFrames];  // int_frame Cp (blood = vb * cp_int for a blood fraction vb)
    float one_minus_vb;
    float pad[3];
};

// Per time boundary (frame start or end) tables of the closed-form tissue integral.
// The voxel-dependent part of int_0^t C_T = K1 (P2(t) - k2 J(t)) is
//   J(t) = A1 J'_1(t) - (A2 + A3) J_1(t) + A2 J_2(t) + A3 J_3(t),
//   J_i(t) = (u_i(t) - v(t)) / (l_i + a),  u_i = t^2 phi2(l_i t),  v = t^2 phi2(-a t),
//   J'_1 = d J_1 / d l_1 = (u'_1 - J_1) / (l_1 + a),  u'_1 = t^3 phi2'(l_1 t),
// with a = k2 + k3.  Near l_i + a = 0 the quotients are replaced by Taylor series in
// d = (-a - l_i) t with coefficients c_k = phi2^(k)(l_i t) / k!.
struct BoundaryRec {
    float t, t2, t3, t4, t5;
    float u[kRates];      // t^2 phi2(l_i t)
    float u1p;            // t^3 phi2'(l_1 t)
    float x[kRates];      // l_i t
    float hsw[kRates];    // switch radius kTaylorR0 + kTaylorR1 |l_i t|
    float coef[kRates][kTaylorCoef];
    float inv_t;          // 1 / t (0 at t = 0)
    float pad;
};

struct KinTab {
    float l[kRates];     // l1, l2, l3
    float w[4];          // A1, -(A2 + A3), A2, A3: weights of J'_1, J_1, J_2, J_3
    int32_t n_bound;     // boundaries actually used
    int32_t i0[kMaxFrames], i1[kMaxFrames];  // boundary index of each frame's start and end
    BoundaryRec b[kMaxBoundaries];
};

// Layout of the constant tables at the start of the caller's workspace.
struct DevTables {
    FrameTab fr;
    KinTab kin;
    // followed by AngleRec[n_ang]
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace kcs
