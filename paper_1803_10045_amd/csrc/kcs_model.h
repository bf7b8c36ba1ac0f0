// Device kinetic model: frame-averaged irreversible two-tissue TAC and its Jacobian, in closed
// form (the time integrals of the model are analytic, Sec. II-C).
//
// With a = k2 + k3 the running tissue integral is int_0^t C_T = K1 (P2(t) - k2 J(t)), where
// P2 is the double integral of the input and J(t) = sum_i w_i J_i(t) is a third divided
// difference of e^{z t} at the points {l_i, 0, 0, -a} (see BoundaryRec).  Every frame value is
//   F_m = [(1 - vb) K1 (dP2_m - k2 dJ_m) + vb dP1_m] / dt_m
// with dP1, dP2 from the host tables and dJ_m = J(t1_m) - J(t0_m).  Derivatives:
//   dF/dK1 = (1 - vb) (dP2 - k2 dJ) / dt,  dF/dk2 = -(1 - vb) K1 (dJ + k2 dJ') / dt,
//   dF/dk3 = -(1 - vb) K1 k2 dJ' / dt,      J' = dJ/da.
#pragma once

#include "kcs_internal.h"

namespace kcs {

// phi2(y) = (e^y - 1 - y) / y^2 and phi2'(y) for y <= 0; inv_y = 1 / y.
template <bool DERIV>
__host__ __device__ __forceinline__ void phi2_pair(float y, float inv_y, float& p2, float& p2d) {
    if (y > -1.0f) {
        // power series: phi2 = sum y^n / (n+2)!, phi2' = sum (n+1) y^n / (n+3)!
        float s = 2.08767569878681e-09f;  // 1/12!
        s = fmaf(s, y, 2.50521083854417e-08f);
        s = fmaf(s, y, 2.75573192239859e-07f);
        s = fmaf(s, y, 2.75573192239859e-06f);
        s = fmaf(s, y, 2.48015873015873e-05f);
        s = fmaf(s, y, 1.98412698412698e-04f);
        s = fmaf(s, y, 1.38888888888889e-03f);
        s = fmaf(s, y, 8.33333333333333e-03f);
        s = fmaf(s, y, 4.16666666666667e-02f);
        s = fmaf(s, y, 1.66666666666667e-01f);
        p2 = fmaf(s, y, 0.5f);
        if (DERIV) {
            float d = 11.0f * 1.60590438368216e-10f;  // (n+1)/(n+3)! for n = 10
            d = fmaf(d, y, 10.0f * 2.08767569878681e-09f);
            d = fmaf(d, y, 9.0f * 2.50521083854417e-08f);
            d = fmaf(d, y, 8.0f * 2.75573192239859e-07f);
            d = fmaf(d, y, 7.0f * 2.75573192239859e-06f);
            d = fmaf(d, y, 6.0f * 2.48015873015873e-05f);
            d = fmaf(d, y, 5.0f * 1.98412698412698e-04f);
            d = fmaf(d, y, 4.0f * 1.38888888888889e-03f);
            d = fmaf(d, y, 3.0f * 8.33333333333333e-03f);
            d = fmaf(d, y, 2.0f * 4.16666666666667e-02f);
            p2d = fmaf(d, y, 1.66666666666667e-01f);
        }
    } else {
        const float e = expf(y);
        const float p1 = (e - 1.0f) * inv_y;
        p2 = (p1 - 1.0f) * inv_y;
        if (DERIV) p2d = (p1 - 2.0f * p2) * inv_y;
    }
}

// p = sum_{j<N} c[j] d^j and (if DERIV) q = dp/dd by Horner's scheme.
template <int N, bool DERIV>
__host__ __device__ __forceinline__ void poly_horner(const float* c, float d, float& p, float& q) {
    p = c[N - 1];
    q = 0.0f;
#pragma unroll
    for (int j = N - 2; j >= 0; --j) {
        if (DERIV) q = (j == N - 2) ? p : fmaf(q, d, p);
        p = fmaf(p, d, c[j]);
    }
}

// Voxel constants of the model.
struct VoxelRates {
    float a, inv_a;
    float inv_b[kRates];  // 1 / (l_i + a)
};

__host__ __device__ __forceinline__ VoxelRates voxel_rates(const KinTab& K, float k2, float k3) {
    VoxelRates v;
    v.a = k2 + k3;
    v.inv_a = 1.0f / v.a;
#pragma unroll
    for (int i = 0; i < kRates; ++i) v.inv_b[i] = 1.0f / (K.l[i] + v.a);
    return v;
}

// J(t) and (if DERIV) dJ/da at one boundary.
template <bool DERIV>
__host__ __device__ __forceinline__ void boundary_J(const KinTab& K, const BoundaryRec& B, const VoxelRates& R, float& J,
                                           float& dJ) {
    const float t = B.t;
    if (t == 0.0f) {
        J = 0.0f;
        dJ = 0.0f;
        return;
    }
    const float y = -R.a * t;
    const float inv_t = B.inv_t;
    float p2, p2d = 0.0f;
    phi2_pair<DERIV>(y, -R.inv_a * inv_t, p2, p2d);
    const float v = B.t2 * p2;
    const float dv = -B.t3 * p2d;  // d v / d a

    float Ji[kRates], dJi[kRates], Jp = 0.0f, dJp = 0.0f;
#pragma unroll
    for (int i = 0; i < kRates; ++i) {
        const float h = B.x[i] - y;  // (l_i + a) t
        if (fabsf(h) >= B.hsw[i]) {
            Ji[i] = (B.u[i] - v) * R.inv_b[i];
            if (DERIV) dJi[i] = -(dv + Ji[i]) * R.inv_b[i];
            if (i == 0) {
                Jp = (B.u1p - Ji[0]) * R.inv_b[0];
                if (DERIV) dJp = -(dJi[0] + Jp) * R.inv_b[0];
            }
        } else {
            // series in d = y - l_i t, with c_k the k-th coefficient (1-based):
            //   J_i = t^3 S(d),  S = sum_{j=0..kTaylor} c_{j+1} d^j,   dJ_i = -t^4 S'(d),
            //   J'_1 = t^4 T(d), T = sum_{j=0..kTaylor} c_{j+2} d^j,   dJ'_1 = -t^5 T'(d);
            // Horner's scheme carries each polynomial's derivative along.
            const float d = -h;
            const float* c = B.coef[i];
            float s, ds;
            poly_horner<kTaylor + 1, DERIV>(c, d, s, ds);
            Ji[i] = B.t3 * s;
            if (DERIV) dJi[i] = -B.t4 * ds;
            if (i == 0) {
                poly_horner<kTaylor + 1, DERIV>(c + 1, d, s, ds);
                Jp = B.t4 * s;
                if (DERIV) dJp = -B.t5 * ds;
            }
        }
    }
    J = K.w[0] * Jp + K.w[1] * Ji[0] + K.w[2] * Ji[1] + K.w[3] * Ji[2];
    if (DERIV) dJ = K.w[0] * dJp + K.w[1] * dJi[0] + K.w[2] * dJi[1] + K.w[3] * dJi[2];
}

// Calls sink(m, F_m, dF/dK1, dF/dk2, dF/dk3, dF/dvb) for every frame m (derivatives 0 when
// !DERIV).  NP = 3: the blood fraction is the study's (FT.one_minus_vb, FT.blood) and vb is
// ignored; NP = 4: it is the voxel's vb (the fourth fitted parameter), and
// dF/dvb = (int_frame Cp - int_frame C_T) / dt.
// UNROLL = false keeps the frame loop rolled, four frames per pass (small code, few registers; the
// sink then sees a run-time frame index and must not index register arrays with it, but m % 4 is
// known in each of the four copies of the body).
template <int M, bool DERIV, bool UNROLL = true, int NP = 3, class Sink>
__host__ __device__ __forceinline__ void model_frames(const FrameTab& FT, const KinTab& K, float K1, float k2, float k3,
                                             float vb, Sink&& sink) {
    static_assert(NP == 3 || NP == 4, "3 or 4 parameters");
    const VoxelRates R = voxel_rates(K, k2, k3);
    const float g = NP == 4 ? 1.0f - vb : FT.one_minus_vb;
    float Jprev = 0.0f, dJprev = 0.0f;
#pragma unroll(UNROLL ? M : 4)
    for (int m = 0; m < M; ++m) {
        if (m == 0 || !FT.contiguous) boundary_J<DERIV>(K, K.b[K.i0[m]], R, Jprev, dJprev);
        float J1, dJ1 = 0.0f;
        boundary_J<DERIV>(K, K.b[K.i1[m]], R, J1, dJ1);
        const float dJ = J1 - Jprev;
        const float tis = FT.dP2[m] - k2 * dJ;
        const float blood = NP == 4 ? vb * FT.cp_int[m] : FT.blood[m];
        const float F = FT.inv_dt[m] * fmaf(g * K1, tis, blood);
        float d0 = 0.0f, d1 = 0.0f, d2 = 0.0f, d3 = 0.0f;
        if (DERIV) {
            const float ddJ = dJ1 - dJprev;
            const float s = g * FT.inv_dt[m];
            d0 = s * tis;
            d1 = -s * K1 * fmaf(k2, ddJ, dJ);
            d2 = -s * K1 * k2 * ddJ;
            if (NP == 4) d3 = FT.inv_dt[m] * (FT.cp_int[m] - K1 * tis);
        }
        sink(m, F, d0, d1, d2, d3);
        Jprev = J1;
        dJprev = dJ1;
    }
}

// m_k(x) = int_0^1 s^k e^{x s} ds for k = 0..kmax (x <= 0), FP64.  Upward recursion
// m_k = (e^x - k m_{k-1}) / x is stable for |x| > k; otherwise the downward recursion
// m_{k-1} = (e^x - x m_k) / k from a high start value given by its power series.
__host__ __device__ inline void moments_fp64(double x, int kmax, double* m) {
    if (x == 0.0) {
        for (int k = 0; k <= kmax; ++k) m[k] = 1.0 / (k + 1);
        return;
    }
    const double e = exp(x);
    if (-x > (double)(kmax + 1)) {
        m[0] = expm1(x) / x;
        for (int k = 1; k <= kmax; ++k) m[k] = (e - k * m[k - 1]) / x;
        return;
    }
    const int K0 = kmax + 60;
    double term = 1.0, acc = 0.0;
    for (int j = 0; j < 400; ++j) {
        acc += term / (double)(j + K0 + 1);
        term *= x / (double)(j + 1);
        if (fabs(term) < 1e-30 * fabs(acc)) break;
    }
    double mk = acc;
    for (int k = K0; k > 0; --k) {
        const double prev = (e - x * mk) / (double)k;
        if (k - 1 <= kmax) m[k - 1] = prev;
        mk = prev;
    }
}

// Boundary record at time t (minutes) for the input-function exponents l[0..2], FP64 -> FP32.
__host__ __device__ inline BoundaryRec make_boundary(double t, const double* l) {
    constexpr int kMom = kTaylorCoef + 1;
    BoundaryRec R;
    R.t = (float)t;
    R.t2 = (float)(t * t);
    R.t3 = (float)(t * t * t);
    R.t4 = (float)(t * t * t * t);
    R.t5 = (float)(t * t * t * t * t);
    double m[kMom + 1];
    for (int i = 0; i < kRates; ++i) {
        const double x = l[i] * t;
        moments_fp64(x, kMom, m);
        R.x[i] = (float)x;
        R.hsw[i] = (float)(kTaylorR0 + kTaylorR1 * fabs(x));
        R.u[i] = (float)(t * t * (m[0] - m[1]));  // t^2 phi2(x), phi2(x) = int_0^1 (1-s) e^{xs} ds
        if (i == 0) R.u1p = (float)(t * t * t * (m[1] - m[2]));  // t^3 phi2'(x)
        double fact = 1.0;
        for (int k = 1; k <= kTaylorCoef; ++k) {
            fact *= k;
            R.coef[i][k - 1] = (float)((m[k] - m[k + 1]) / fact);  // phi2^(k)(x) / k!
        }
    }
    R.inv_t = R.t > 0.0f ? 1.0f / R.t : 0.0f;
    R.pad = 0.0f;
    return R;
}

}  // namespace kcs
