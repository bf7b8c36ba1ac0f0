// K-lm: one synchronous MAP Levenberg-Marquardt iteration (Eq. 4-7), one thread per voxel.
//
// Per voxel: model TAC F and its 3 Jacobian columns from the closed form (frame by frame,
// accumulating J^T J and J^T r on the fly, so no Jacobian is stored), the Huber neighbour
// gradient over the in-plane 8-neighbourhood of the previous maps (Jacobi update, all voxels see
// the same old neighbours; a workgroup stages its tile of the maps with a one-voxel border in LDS
// once, and both Huber evaluations read it there), the damped 3x3 normal equations solved by a
// diagonally scaled Cholesky factorisation in registers, box clipping, and the accept test on
// the change of the voxel objective,
//   dPhi = (r'^T r' - r^T r) / 2 + beta_h (E(xi') - E(xi)),   r = x - F(xi), r' = x - F(xi').
// The data terms depend only on the voxel's own maps and image, so the normal equations at the
// trial maps, evaluated with the Jacobian, are those of the next iteration whenever the step is
// accepted, and those at the current maps stay valid when it is rejected.  A fit therefore
// carries J^T J, J^T r and r^T r from one iteration to the next in a per-voxel state buffer: its
// first iteration evaluates the model twice (with the Jacobian at the current and the trial
// maps), the others once (at the trial maps, with the Jacobian unless it is the fit's last).
#include "kcs_device.h"
#include "kcs_launch.h"
#include "kcs_model.h"

namespace kcs {

constexpr int kLmThreads = 256;

__host__ __device__ __forceinline__ float huber(float t, float d) {
    const float at = fabsf(t);
    return at <= d ? 0.5f * t * t : d * at - 0.5f * d * d;
}

// The maps of a workgroup's voxel tile with a one-voxel border, staged in LDS: for each staged
// plane (the voxel's own, and with the 3x3x3 neighbourhood the planes below and above, slots 0 to
// 2 from below), (TY + 2) rows of (TX + 2) voxels, the NP maps of a voxel adjacent; the tile's
// voxel (i, j) sits at row j - j0 + 1, column i - i0 + 1.  Entries outside the image are not
// written and never read.
constexpr int kHaloMaxTile = 66 * 6;  // (TX + 2)(TY + 2) at most, over TX in {8, 16, 32, 64}, TY = 256 / TX

// Weighted Huber energy sum_k w_k sum_p H(q_p - xi_kp) over the neighbours k of voxel (i, j, z)
// in the NP maps xi (neighbours outside the image dropped), and the gradient terms
// psi_p = sum_k w_k clip(q_p - xi_kp, -delta_p, delta_p).  The neighbours are the 8 in-plane ones
// (weights 1 and 1/sqrt(2)) and, with a.nbr3d, the 18 of the planes z - 1 and z + 1 (weights
// a.w_plane by the number of in-plane offsets).
// Adds the terms of the 3x3 neighbours in plane zz of voxel (i, j) (the voxel itself skipped when
// zz is its own plane); w_edge, w_diag weight neighbours with one and two in-plane offsets.
// corner: the staged maps of voxel (i - 1, j - 1) in plane zz; w: staged voxels per row.
template <int NP>
__device__ __forceinline__ void plane_terms(const float* corner, int w, const LmArgs& a, int i, int j, bool own,
                                            float w_centre, float w_edge, float w_diag, const float (&q)[NP], float& e,
                                            float (&psi)[NP]) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const float* row = corner + (dy + 1) * w * NP;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (own && dy == 0 && dx == 0) continue;
            const int jj = j + dy, ii = i + dx;
            if (jj < 0 || jj >= a.ny || ii < 0 || ii >= a.nx) continue;
            const int off = (dx != 0) + (dy != 0);
            const float wk = off == 0 ? w_centre : (off == 1 ? w_edge : w_diag);
            float h = 0.0f;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const float d = q[p] - row[(dx + 1) * NP + p];
                psi[p] += wk * fminf(fmaxf(d, -a.delta[p]), a.delta[p]);
                h = p == 0 ? huber(d, a.delta[p]) : h + huber(d, a.delta[p]);
            }
            e += wk * h;
        }
    }
}

// own: the staged maps of voxel (i - 1, j - 1) in the voxel's own plane; plane_step: staged
// values per plane.
template <int NP, bool NBR3D>
__device__ __forceinline__ float neighbour_energy(const float* own, int w, int plane_step, const LmArgs& a, int i,
                                                  int j, int z, const float (&q)[NP], float (&psi)[NP]) {
    float e = 0.0f;
#pragma unroll
    for (int p = 0; p < NP; ++p) psi[p] = 0.0f;
    plane_terms<NP>(own, w, a, i, j, true, 0.0f, 1.0f, 0.70710678118654752f, q, e, psi);
    if (NBR3D) {
#pragma unroll 1
        for (int dz = -1; dz <= 1; dz += 2) {
            if (z + dz < 0 || z + dz >= a.nz) continue;
            plane_terms<NP>(own + dz * plane_step, w, a, i, j, false, a.w_plane[0], a.w_plane[1], a.w_plane[2], q, e,
                            psi);
        }
    }
    return e;
}

// Frame m of a voxel's image record read four frames at a time: the lanes of a wave read records
// M floats apart, so a load of one float per lane touches as many cache lines as a load of four.
// Called with m = 0, 1, ..., M - 1 in order from the frame loop of model_frames, which is unrolled
// by four, so m % 4 is a constant in every call and the selects fold away.
template <int M>
struct RecordReader {
    static_assert(M % 4 == 0, "frames must be a multiple of 4");
    const float4* p;  // the record, 16-byte aligned
    float4 q;
    __host__ __device__ __forceinline__ float operator()(int m) {
        if ((m & 3) == 0) q = p[m >> 2];
        const int k = m & 3;
        return k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
    }
};

// Normal equations of the data term at maps xi: J^T J (packed lower triangle, row by row:
// A[r(r+1)/2 + c] for c <= r), J^T r (g) and r^T r (rr).  NP(NP + 1)/2 + NP + 1 floats: the
// per-voxel state a fit carries between iterations (10 for 3 maps, 15 for 4).
template <int NP>
struct Normal {
    static constexpr int kTri = NP * (NP + 1) / 2;
    static constexpr int kFloats = kTri + NP + 1;
    float A[kTri];
    float g[NP];
    float rr;
};

__host__ __device__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

template <int M, int NP>
__host__ __device__ __forceinline__ Normal<NP> normal_equations(const FrameTab& fr, const KinTab& K, const float* xv,
                                                                const float (&xi)[NP]) {
    Normal<NP> n;
#pragma unroll
    for (int k = 0; k < Normal<NP>::kTri; ++k) n.A[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < NP; ++k) n.g[k] = 0.0f;
    n.rr = 0.0f;
    RecordReader<M> xr{reinterpret_cast<const float4*>(xv), {}};
    model_frames<M, true, false, NP>(fr, K, xi[0], xi[1], xi[2], NP == 4 ? xi[NP - 1] : 0.0f,
                                     [&](int m, float F, float j0, float j1, float j2, float j3) {
                                         const float jv[4] = {j0, j1, j2, j3};
                                         const float r = xr(m) - F;
#pragma unroll
                                         for (int rw = 0; rw < NP; ++rw)
#pragma unroll
                                             for (int c = 0; c <= rw; ++c)
                                                 n.A[tri(rw, c)] = fmaf(jv[rw], jv[c], n.A[tri(rw, c)]);
#pragma unroll
                                         for (int k = 0; k < NP; ++k) n.g[k] = fmaf(jv[k], r, n.g[k]);
                                         n.rr = fmaf(r, r, n.rr);
                                     });
    return n;
}

// r^T r of the data term at maps xi, from the model without its Jacobian.  F and the sum are
// formed by the same operations as in normal_equations, so the two round identically.
template <int M, int NP>
__host__ __device__ __forceinline__ float residual_norm(const FrameTab& fr, const KinTab& K, const float* xv,
                                                        const float (&xi)[NP]) {
    float rr = 0.0f;
    RecordReader<M> xr{reinterpret_cast<const float4*>(xv), {}};
    model_frames<M, false, false, NP>(fr, K, xi[0], xi[1], xi[2], NP == 4 ? xi[NP - 1] : 0.0f,
                                      [&](int m, float F, float, float, float, float) {
                                          const float r = xr(m) - F;
                                          rr = fmaf(r, r, rr);
                                      });
    return rr;
}

template <int NP>
__host__ __device__ __forceinline__ Normal<NP> load_normal(const float* __restrict__ st, size_t N, size_t v) {
    Normal<NP> n;
#pragma unroll
    for (int k = 0; k < Normal<NP>::kTri; ++k) n.A[k] = st[k * N + v];
#pragma unroll
    for (int k = 0; k < NP; ++k) n.g[k] = st[(Normal<NP>::kTri + k) * N + v];
    n.rr = st[(Normal<NP>::kFloats - 1) * N + v];
    return n;
}

template <int NP>
__host__ __device__ __forceinline__ void store_normal(float* __restrict__ st, size_t N, size_t v, const Normal<NP>& n) {
#pragma unroll
    for (int k = 0; k < Normal<NP>::kTri; ++k) st[k * N + v] = n.A[k];
#pragma unroll
    for (int k = 0; k < NP; ++k) st[(Normal<NP>::kTri + k) * N + v] = n.g[k];
    st[(Normal<NP>::kFloats - 1) * N + v] = n.rr;
}

// xi_in: the staged maps of voxel (i - 1, j - 1) in the voxel's own plane (see kHaloMaxTile);
// w: staged voxels per row; plane_step: staged values per plane.
template <int M, int NP, bool NBR3D>
__device__ __forceinline__ void lm_voxel(const KinTab* __restrict__ K, const float* __restrict__ x, const float* xi_in,
                                         int w, int plane_step, float* __restrict__ xi_out, float* __restrict__ lam_io,
                                         float* __restrict__ state, const LmArgs& a, int i, int j, int z) {
    const size_t plane = (size_t)a.nx * a.ny;
    const size_t N = plane * a.nz;
    const size_t v = (size_t)z * plane + (size_t)j * a.nx + i;

    const float* xv = x + v * M;
    float p[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) p[k] = xi_in[(w + 1) * NP + k];

    // Huber terms over the neighbours of the previous maps: psi (gradient) and e0 (energy) at the
    // current parameters.  The neighbours are read again from LDS for the trial energy below
    // instead of being held in registers through the model evaluations.
    float psi[NP];
    const float e0 = neighbour_energy<NP, NBR3D>(xi_in, w, plane_step, a, i, j, z, p, psi);
    // data-term normal equations at the current parameters
    const Normal<NP> n0 = a.have_state ? load_normal<NP>(state, N, v) : normal_equations<M, NP>(a.fr, *K, xv, p);
    float g[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) g[k] = n0.g[k] - a.beta_h * psi[k];

    float lam = a.reset_lambda ? 0.0f : lam_io[v];
    if (!(lam > 0.0f)) {
        float dmax = n0.A[tri(NP - 1, NP - 1)];
#pragma unroll
        for (int k = NP - 2; k >= 0; --k) dmax = fmaxf(n0.A[tri(k, k)], dmax);
        lam = a.tau * dmax;
    }

    // (A + lam I) step = g, symmetrically scaled by the inverse square roots of the diagonal,
    // then a Cholesky factorisation in registers
    float sc[NP], B[Normal<NP>::kTri], L[Normal<NP>::kTri];
#pragma unroll
    for (int k = 0; k < NP; ++k) sc[k] = 1.0f / sqrtf(n0.A[tri(k, k)] + lam);
#pragma unroll
    for (int r = 0; r < NP; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c)
            B[tri(r, c)] = c == r ? (n0.A[tri(r, r)] + lam) * sc[r] * sc[r] : n0.A[tri(r, c)] * sc[c] * sc[r];
#pragma unroll
    for (int r = 0; r < NP; ++r) {
#pragma unroll
        for (int c = 0; c < r; ++c) {
            float acc = B[tri(r, c)];
#pragma unroll
            for (int k = 0; k < c; ++k) acc = acc - L[tri(r, k)] * L[tri(c, k)];
            L[tri(r, c)] = acc / L[tri(c, c)];
        }
        float acc = B[tri(r, r)];
#pragma unroll
        for (int k = 0; k < r; ++k) acc = acc - L[tri(r, k)] * L[tri(r, k)];
        L[tri(r, r)] = r == 0 ? sqrtf(acc) : sqrtf(fmaxf(acc, 1e-30f));
    }
    float y[NP], zz[NP];
#pragma unroll
    for (int r = 0; r < NP; ++r) {
        float acc = g[r] * sc[r];
#pragma unroll
        for (int k = 0; k < r; ++k) acc = acc - L[tri(r, k)] * y[k];
        y[r] = acc / L[tri(r, r)];
    }
#pragma unroll
    for (int r = NP - 1; r >= 0; --r) {
        float acc = y[r];
#pragma unroll
        for (int k = r + 1; k < NP; ++k) acc = acc - L[tri(k, r)] * zz[k];
        zz[r] = acc / L[tri(r, r)];
    }
    float q[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) q[k] = fminf(fmaxf(p[k] + zz[k] * sc[k], a.lo[k]), a.hi[k]);

    float unused[NP];
    const float e1 = neighbour_energy<NP, NBR3D>(xi_in, w, plane_step, a, i, j, z, q, unused);

    // data term at the trial parameters, with its normal equations when another iteration follows
    // (they are the next iteration's if the step is kept); the last iteration of a fit needs only
    // r'^T r', which rounds like the normal equations' own, so a fit of n iterations still rounds
    // exactly like n calls of one iteration each.
    Normal<NP> n1;
    float rr1;
    if (a.need_state) {
        n1 = normal_equations<M, NP>(a.fr, *K, xv, q);
        rr1 = n1.rr;
    } else {
        rr1 = residual_norm<M, NP>(a.fr, *K, xv, q);
    }
    const float dphi = fmaf(a.beta_h, e1 - e0, 0.5f * (rr1 - n0.rr));
    const float phi0 = fmaf(a.beta_h, e0, 0.5f * n0.rr);
    const bool accept = dphi < -a.eta * phi0;
#pragma unroll
    for (int k = 0; k < NP; ++k) xi_out[k * N + v] = accept ? q[k] : p[k];
    lam_io[v] = accept ? fmaxf(lam * 0.1f, a.lam_min) : fminf(lam * 10.0f, a.lam_max);
    // the state holds the normal equations of the maps this iteration leaves
    if (a.need_state) {
        if (accept) store_normal<NP>(state, N, v, n1);
        else if (!a.have_state) store_normal<NP>(state, N, v, n0);
    }
}

// Width of the voxel tile of a workgroup (tile_x x 256 / tile_x voxels, one per thread): of 64,
// 32, 16 and 8, the one that pads the plane least (idle lanes cost a whole lane's model
// evaluations), the wider on a tie (a wavefront then reads longer contiguous runs of the image).
// The tile does not change any voxel's result.
int lm_tile_x(int nx, int ny) {
    int best = 64;
    long best_area = -1;
    for (int tx : {64, 32, 16, 8}) {
        const int ty = kLmThreads / tx;
        const long area = (long)((nx + tx - 1) / tx * tx) * ((ny + ty - 1) / ty * ty);
        if (best_area < 0 || area < best_area) {
            best = tx;
            best_area = area;
        }
    }
    return best;
}

uint32_t lm_groups(int nx, int ny, int nz, int tile_x) {
    const int ty = kLmThreads / tile_x;
    return (uint32_t)((nx + tile_x - 1) / tile_x) * ((ny + ty - 1) / ty) * nz;
}

template <int M, int NP, bool NBR3D, class Src>
__global__ __launch_bounds__(kLmThreads) void klm_kernel(Src src) {
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const LmJob& J = src.find(w);
    const LmArgs& a = J.a;
    const uint32_t lw = w - J.w0;
    const int TX = a.tile_x, TY = kLmThreads / TX, sx = __builtin_ctz((unsigned)TX);  // TX a power of 2
    const uint32_t tx = (a.nx + TX - 1) >> sx, ty = (a.ny + TY - 1) / TY;
    const int z = lw / (tx * ty);
    const uint32_t rr = lw % (tx * ty);
    const int j0 = (rr / tx) * TY, i0 = (rr % tx) * TX;
    const int j = j0 + (threadIdx.x >> sx);
    const int i = i0 + (threadIdx.x & (TX - 1));
    if (z >= a.nz) return;  // the whole workgroup: its tiles are past the last plane
    // stage the previous maps of the tile and its border (and of the neighbouring planes) in LDS
    constexpr int NPL = NBR3D ? 3 : 1;
    __shared__ float halo[NPL * kHaloMaxTile * NP];
    const int hw = TX + 2, n_tile = hw * (TY + 2);
    const size_t plane = (size_t)a.nx * a.ny, N = plane * a.nz;
    for (int e = threadIdx.x; e < NPL * n_tile; e += kLmThreads) {
        const int slot = e / n_tile, t = e - slot * n_tile;
        const int zz = z + (NPL == 1 ? 0 : slot - 1);
        const int r = t / hw, c = t - r * hw;
        const int jj = j0 - 1 + r, ii = i0 - 1 + c;
        if (zz >= 0 && zz < a.nz && jj >= 0 && jj < a.ny && ii >= 0 && ii < a.nx) {
            const size_t u = (size_t)zz * plane + (size_t)jj * a.nx + ii;
#pragma unroll
            for (int p = 0; p < NP; ++p) halo[e * NP + p] = J.xi_in[p * N + u];
        }
    }
    __syncthreads();
    if (i >= a.nx || j >= a.ny) return;
    // the staged maps of voxel (i - 1, j - 1) in the voxel's own plane (slot 1 of 3, or 0 of 1)
    const float* corner = halo + (((NPL == 1 ? 0 : 1) * (TY + 2) + (j - j0)) * hw + (i - i0)) * NP;
    lm_voxel<M, NP, NBR3D>(J.K, J.x, corner, hw, n_tile * NP, J.xi_out, J.lam, J.state, a, i, j, z);
}

// All jobs of one launch share the neighbourhood (nbr3d) and the number of fitted maps (np), so
// that the in-plane three-map kernel carries no code or registers for the other cases.
template <int NP, bool NBR3D, class Src>
static hipError_t dispatch_lm_m(int M, Src src, uint32_t groups, hipStream_t st) {
    const dim3 g(xcd_round_up(groups)), b(kLmThreads);
    switch (M) {
        case 8: hipLaunchKernelGGL((klm_kernel<8, NP, NBR3D, Src>), g, b, 0, st, src); break;
        case 16: hipLaunchKernelGGL((klm_kernel<16, NP, NBR3D, Src>), g, b, 0, st, src); break;
        case 24: hipLaunchKernelGGL((klm_kernel<24, NP, NBR3D, Src>), g, b, 0, st, src); break;
        case 32: hipLaunchKernelGGL((klm_kernel<32, NP, NBR3D, Src>), g, b, 0, st, src); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class Src>
static hipError_t dispatch_lm(int M, int np, bool nbr3d, Src src, uint32_t groups, hipStream_t st) {
    if (np == 4)
        return nbr3d ? dispatch_lm_m<4, true>(M, src, groups, st) : dispatch_lm_m<4, false>(M, src, groups, st);
    if (np == 3)
        return nbr3d ? dispatch_lm_m<3, true>(M, src, groups, st) : dispatch_lm_m<3, false>(M, src, groups, st);
    return hipErrorInvalidValue;
}

hipError_t launch_lm(int M, const KinTab* K, const float* x, const float* xi_in, float* xi_out, float* lam,
                     float* state, const LmArgs& a, hipStream_t st) {
    OneJob<LmJob> src{LmJob{a, K, x, xi_in, xi_out, lam, state, 0}};
    return dispatch_lm(M, a.np, a.nbr3d != 0, src, lm_groups(a.nx, a.ny, a.nz, a.tile_x), st);
}

hipError_t launch_lm_jobs(int M, bool nbr3d, JobTable<LmJob> jobs, uint32_t groups, hipStream_t st) {
    // plans fit three maps
    return nbr3d ? dispatch_lm_m<3, true>(M, jobs, groups, st) : dispatch_lm_m<3, false>(M, jobs, groups, st);
}

}  // namespace kcs
