// K-lm: one synchronous MAP Levenberg-Marquardt iteration (Eq. 4-7), one thread per voxel.
//
// Per voxel: model TAC F and its 3 Jacobian columns from the closed form (frame by frame,
// accumulating J^T J and J^T r on the fly, so no Jacobian is stored), the Huber neighbour
// gradient over the in-plane 8-neighbourhood read from the previous maps (Jacobi update, all
// voxels see the same old neighbours), the damped 3x3 normal equations solved by a
// diagonally scaled Cholesky factorisation in registers, box clipping, and the accept test on
// the change of the voxel objective,
//   dPhi = (r'^T r' - r^T r) / 2 + beta_h (E(xi') - E(xi)),   r = x - F(xi), r' = x - F(xi').
// The data terms depend only on the voxel's own maps and image, so the normal equations at the
// trial maps, evaluated with the Jacobian, are those of the next iteration whenever the step is
// accepted, and those at the current maps stay valid when it is rejected.  A fit therefore
// carries J^T J, J^T r and r^T r from one iteration to the next in a per-voxel state buffer: its
// first iteration evaluates the model twice (with the Jacobian at the current and the trial
// maps), the others once (with the Jacobian, at the trial maps).
#include "kcs_device.h"
#include "kcs_launch.h"
#include "kcs_model.h"

namespace kcs {

constexpr int kLmTileX = 64, kLmTileY = 4;

__host__ __device__ __forceinline__ float huber(float t, float d) {
    const float at = fabsf(t);
    return at <= d ? 0.5f * t * t : d * at - 0.5f * d * d;
}

// Weighted Huber energy sum_k w_k sum_p H(q_p - xi_kp) over the neighbours k of voxel (i, j, z)
// in the maps xi (neighbours outside the image dropped), and the gradient terms
// psi_p = sum_k w_k clip(q_p - xi_kp, -delta_p, delta_p).  The neighbours are the 8 in-plane ones
// (weights 1 and 1/sqrt(2)) and, with a.nbr3d, the 18 of the planes z - 1 and z + 1 (weights
// a.w_plane by the number of in-plane offsets).
// Adds the terms of the 3x3 neighbours in plane zz of voxel (i, j) (the voxel itself skipped when
// zz is its own plane); w_edge, w_diag weight neighbours with one and two in-plane offsets.
__host__ __device__ __forceinline__ void plane_terms(const float* __restrict__ xi, const LmArgs& a, int i, int j,
                                                     int zz, bool own, float w_centre, float w_edge, float w_diag,
                                                     size_t N, float q0, float q1, float q2, float& e,
                                                     float (&psi)[3]) {
    const size_t plane = (size_t)a.nx * a.ny;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (own && dy == 0 && dx == 0) continue;
            const int jj = j + dy, ii = i + dx;
            if (jj < 0 || jj >= a.ny || ii < 0 || ii >= a.nx) continue;
            const size_t u = (size_t)zz * plane + (size_t)jj * a.nx + ii;
            const int off = (dx != 0) + (dy != 0);
            const float w = off == 0 ? w_centre : (off == 1 ? w_edge : w_diag);
            const float d0 = q0 - xi[u], d1 = q1 - xi[N + u], d2 = q2 - xi[2 * N + u];
            psi[0] += w * fminf(fmaxf(d0, -a.delta[0]), a.delta[0]);
            psi[1] += w * fminf(fmaxf(d1, -a.delta[1]), a.delta[1]);
            psi[2] += w * fminf(fmaxf(d2, -a.delta[2]), a.delta[2]);
            e += w * (huber(d0, a.delta[0]) + huber(d1, a.delta[1]) + huber(d2, a.delta[2]));
        }
    }
}

template <bool NBR3D>
__host__ __device__ __forceinline__ float neighbour_energy(const float* __restrict__ xi, const LmArgs& a, int i, int j,
                                                           int z, size_t N, float q0, float q1, float q2,
                                                           float (&psi)[3]) {
    float e = 0.0f;
    psi[0] = psi[1] = psi[2] = 0.0f;
    plane_terms(xi, a, i, j, z, true, 0.0f, 1.0f, 0.70710678118654752f, N, q0, q1, q2, e, psi);
    if (NBR3D) {
#pragma unroll 1
        for (int dz = -1; dz <= 1; dz += 2) {
            if (z + dz < 0 || z + dz >= a.nz) continue;
            plane_terms(xi, a, i, j, z + dz, false, a.w_plane[0], a.w_plane[1], a.w_plane[2], N, q0, q1, q2, e, psi);
        }
    }
    return e;
}

// Normal equations of the data term at maps (k1, k2, k3): J^T J (A), J^T r (g) and r^T r (rr).
struct Normal {
    float A00, A01, A02, A11, A12, A22, g0, g1, g2, rr;
};

template <int M>
__host__ __device__ __forceinline__ Normal normal_equations(const FrameTab& fr, const KinTab& K, const float* xv,
                                                            float k1, float k2, float k3) {
    Normal n{0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    model_frames<M, true, false>(fr, K, k1, k2, k3, [&](int m, float F, float j0, float j1, float j2) {
        const float r = xv[m] - F;
        n.A00 = fmaf(j0, j0, n.A00);
        n.A01 = fmaf(j0, j1, n.A01);
        n.A02 = fmaf(j0, j2, n.A02);
        n.A11 = fmaf(j1, j1, n.A11);
        n.A12 = fmaf(j1, j2, n.A12);
        n.A22 = fmaf(j2, j2, n.A22);
        n.g0 = fmaf(j0, r, n.g0);
        n.g1 = fmaf(j1, r, n.g1);
        n.g2 = fmaf(j2, r, n.g2);
        n.rr = fmaf(r, r, n.rr);
    });
    return n;
}

__host__ __device__ __forceinline__ Normal load_normal(const float* __restrict__ st, size_t N, size_t v) {
    return Normal{st[v], st[N + v], st[2 * N + v], st[3 * N + v], st[4 * N + v],
                  st[5 * N + v], st[6 * N + v], st[7 * N + v], st[8 * N + v], st[9 * N + v]};
}

__host__ __device__ __forceinline__ void store_normal(float* __restrict__ st, size_t N, size_t v, const Normal& n) {
    st[v] = n.A00;
    st[N + v] = n.A01;
    st[2 * N + v] = n.A02;
    st[3 * N + v] = n.A11;
    st[4 * N + v] = n.A12;
    st[5 * N + v] = n.A22;
    st[6 * N + v] = n.g0;
    st[7 * N + v] = n.g1;
    st[8 * N + v] = n.g2;
    st[9 * N + v] = n.rr;
}

template <int M, bool NBR3D>
__host__ __device__ __forceinline__ void lm_voxel(const KinTab* __restrict__ K, const float* __restrict__ x,
                                                  const float* __restrict__ xi_in, float* __restrict__ xi_out,
                                                  float* __restrict__ lam_io, float* __restrict__ state,
                                                  const LmArgs& a, int i, int j, int z) {
    const size_t plane = (size_t)a.nx * a.ny;
    const size_t N = plane * a.nz;
    const size_t v = (size_t)z * plane + (size_t)j * a.nx + i;

    const float* xv = x + v * M;
    const float p0 = xi_in[v], p1 = xi_in[N + v], p2 = xi_in[2 * N + v];

    // Huber terms over the neighbours of the previous maps: psi (gradient) and e0 (energy) at the
    // current parameters.  The neighbours are read again for the trial energy below instead of
    // being held in registers through the model evaluations (they are cache hits).
    float psi[3] = {0.0f, 0.0f, 0.0f};
    const float e0 = neighbour_energy<NBR3D>(xi_in, a, i, j, z, N, p0, p1, p2, psi);
    // data-term normal equations at the current parameters
    const Normal n0 = a.have_state ? load_normal(state, N, v) : normal_equations<M>(a.fr, *K, xv, p0, p1, p2);
    const float A00 = n0.A00, A01 = n0.A01, A02 = n0.A02, A11 = n0.A11, A12 = n0.A12, A22 = n0.A22;
    const float g0 = n0.g0 - a.beta_h * psi[0];
    const float g1 = n0.g1 - a.beta_h * psi[1];
    const float g2 = n0.g2 - a.beta_h * psi[2];

    float lam = a.reset_lambda ? 0.0f : lam_io[v];
    if (!(lam > 0.0f)) lam = a.tau * fmaxf(A00, fmaxf(A11, A22));

    // (A + lam I) step = g, symmetrically scaled by the inverse square roots of the diagonal,
    // then a Cholesky factorisation in registers
    const float s0 = 1.0f / sqrtf(A00 + lam), s1 = 1.0f / sqrtf(A11 + lam), s2 = 1.0f / sqrtf(A22 + lam);
    const float B00 = (A00 + lam) * s0 * s0, B11 = (A11 + lam) * s1 * s1, B22 = (A22 + lam) * s2 * s2;
    const float B01 = A01 * s0 * s1, B02 = A02 * s0 * s2, B12 = A12 * s1 * s2;
    const float L00 = sqrtf(B00);
    const float L10 = B01 / L00, L20 = B02 / L00;
    const float L11 = sqrtf(fmaxf(B11 - L10 * L10, 1e-30f));
    const float L21 = (B12 - L20 * L10) / L11;
    const float L22 = sqrtf(fmaxf(B22 - L20 * L20 - L21 * L21, 1e-30f));
    const float y0 = g0 * s0 / L00;
    const float y1 = (g1 * s1 - L10 * y0) / L11;
    const float y2 = (g2 * s2 - L20 * y0 - L21 * y1) / L22;
    const float z2 = y2 / L22;
    const float z1 = (y1 - L21 * z2) / L11;
    const float z0 = (y0 - L10 * z1 - L20 * z2) / L00;
    const float q0 = fminf(fmaxf(p0 + z0 * s0, a.lo[0]), a.hi[0]);
    const float q1 = fminf(fmaxf(p1 + z1 * s1, a.lo[1]), a.hi[1]);
    const float q2 = fminf(fmaxf(p2 + z2 * s2, a.lo[2]), a.hi[2]);

    float unused[3];
    const float e1 = neighbour_energy<NBR3D>(xi_in, a, i, j, z, N, q0, q1, q2, unused);

    // data term at the trial parameters, with its normal equations (the next iteration's when
    // the step is kept).  The last iteration of a fit needs only r'^T r', but evaluating it the
    // same way in every iteration makes a fit of n iterations round exactly like n calls of one
    // iteration each, whatever the call pattern.
    const Normal n1 = normal_equations<M>(a.fr, *K, xv, q0, q1, q2);
    const float dphi = fmaf(a.beta_h, e1 - e0, 0.5f * (n1.rr - n0.rr));
    const float phi0 = fmaf(a.beta_h, e0, 0.5f * n0.rr);
    const bool accept = dphi < -a.eta * phi0;
    xi_out[v] = accept ? q0 : p0;
    xi_out[N + v] = accept ? q1 : p1;
    xi_out[2 * N + v] = accept ? q2 : p2;
    lam_io[v] = accept ? fmaxf(lam * 0.1f, a.lam_min) : fminf(lam * 10.0f, a.lam_max);
    // the state holds the normal equations of the maps this iteration leaves
    if (a.need_state) {
        if (accept) store_normal(state, N, v, n1);
        else if (!a.have_state) store_normal(state, N, v, n0);
    }
}

uint32_t lm_groups(int nx, int ny, int nz) {
    return (uint32_t)((nx + kLmTileX - 1) / kLmTileX) * ((ny + kLmTileY - 1) / kLmTileY) * nz;
}

template <int M, bool NBR3D, class Src>
__global__ __launch_bounds__(256) void klm_kernel(Src src) {
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const LmJob& J = src.find(w);
    const LmArgs& a = J.a;
    const uint32_t lw = w - J.w0;
    const uint32_t tx = (a.nx + kLmTileX - 1) / kLmTileX, ty = (a.ny + kLmTileY - 1) / kLmTileY;
    const int z = lw / (tx * ty);
    const uint32_t rr = lw % (tx * ty);
    const int j = (rr / tx) * kLmTileY + threadIdx.x / kLmTileX;
    const int i = (rr % tx) * kLmTileX + threadIdx.x % kLmTileX;
    if (z >= a.nz || i >= a.nx || j >= a.ny) return;
    lm_voxel<M, NBR3D>(J.K, J.x, J.xi_in, J.xi_out, J.lam, J.state, a, i, j, z);
}

// All jobs of one launch share the neighbourhood (nbr3d), so that the in-plane kernel carries no
// code or registers for the 3x3x3 case.
template <bool NBR3D, class Src>
static hipError_t dispatch_lm_m(int M, Src src, uint32_t groups, hipStream_t st) {
    const dim3 g(xcd_round_up(groups)), b(kLmTileX * kLmTileY);
    switch (M) {
        case 8: hipLaunchKernelGGL((klm_kernel<8, NBR3D, Src>), g, b, 0, st, src); break;
        case 16: hipLaunchKernelGGL((klm_kernel<16, NBR3D, Src>), g, b, 0, st, src); break;
        case 24: hipLaunchKernelGGL((klm_kernel<24, NBR3D, Src>), g, b, 0, st, src); break;
        case 32: hipLaunchKernelGGL((klm_kernel<32, NBR3D, Src>), g, b, 0, st, src); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class Src>
static hipError_t dispatch_lm(int M, bool nbr3d, Src src, uint32_t groups, hipStream_t st) {
    return nbr3d ? dispatch_lm_m<true>(M, src, groups, st) : dispatch_lm_m<false>(M, src, groups, st);
}

hipError_t launch_lm(int M, const KinTab* K, const float* x, const float* xi_in, float* xi_out, float* lam,
                     float* state, const LmArgs& a, hipStream_t st) {
    OneJob<LmJob> src{LmJob{a, K, x, xi_in, xi_out, lam, state, 0}};
    return dispatch_lm(M, a.nbr3d != 0, src, lm_groups(a.nx, a.ny, a.nz), st);
}

hipError_t launch_lm_jobs(int M, bool nbr3d, JobTable<LmJob> jobs, uint32_t groups, hipStream_t st) {
    return dispatch_lm(M, nbr3d, jobs, groups, st);
}

}  // namespace kcs
