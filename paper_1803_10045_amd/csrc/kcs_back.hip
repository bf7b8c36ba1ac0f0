// K-back: voxel-driven (gather) back projector and the fused OS-MAP-OSL-KP update.
//
// One thread per voxel.  For each angle of the subset the voxel's footprint on the detector
// covers at most ceil(2 w1 / du) + 1 bins; the exact intersection length of each bin's ray with
// the voxel square (the pixel chord, identical to the Siddon length of that ray in that pixel)
// weights the bin's M-frame record.  The gather needs no atomics and no transposed system
// matrix; the subset's angle constants are built once per workgroup in LDS.
//
// OSL update (Eq. 2 with the kinetics-derived potential of Eq. 3, sigma^2 = F / n):
//   x_new = x * b / D,  b = E_m sum_d p_vd q_dm,  D = n_m (1 + beta (x - F) / max(F, eps_F)),
//   n_m = E_m sum_d p_vd;  E_m cancels between b and D.  x is kept where sum_d p_vd = 0.
// F, the model TAC of the current kinetic maps, does not change during an OSL pass; it is
// evaluated once per pass (kcs_model pass) and read here.
#include "kcs_device.h"
#include "kcs_launch.h"

namespace kcs {

constexpr int kTileX = 64, kTileY = 4;
constexpr int kMaxSubsetAngles = 1024;

struct TileIdx {
    int i, j, z;
    bool valid;
};

__device__ __forceinline__ TileIdx tile_voxel(uint32_t w, int nx, int ny, int nz) {
    const uint32_t tx = (nx + kTileX - 1) / kTileX, ty = (ny + kTileY - 1) / kTileY;
    TileIdx t;
    t.z = w / (tx * ty);
    const uint32_t r = w % (tx * ty);
    t.j = (r / tx) * kTileY + threadIdx.x / kTileX;
    t.i = (r % tx) * kTileX + threadIdx.x % kTileX;
    t.valid = t.z < nz && t.i < nx && t.j < ny;
    return t;
}

uint32_t voxel_tile_groups(int nx, int ny, int nz) {
    const uint32_t tx = (nx + kTileX - 1) / kTileX, ty = (ny + kTileY - 1) / kTileY;
    return tx * ty * (uint32_t)nz;
}

// Builds the subset's angle constants in LDS; all threads of the block take part.
__device__ __forceinline__ void subset_angles_to_lds(AngleRec* sA, const ProjArgs& p) {
    for (int al = threadIdx.x; al < p.A_q; al += blockDim.x) sA[al] = make_angle(p.q + al * p.Q, p.n_ang, p.ang0, p.h);
    __syncthreads();
}

// acc_m = sum_{d in S_q} p_vd y_dm and sens = sum_{d in S_q} p_vd for voxel (i, j, z).
template <int M>
__host__ __device__ __forceinline__ void gather(const AngleRec* sA, const ProjArgs& p, const float* __restrict__ y, int i, int j,
                                       int z, float (&acc)[M], float& sens) {
    const float xc = ((float)i - 0.5f * (float)(p.nx - 1)) * p.h;
    const float yc = ((float)j - 0.5f * (float)(p.ny - 1)) * p.h;
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0f;
    sens = 0.0f;
    const float* yz = y + (size_t)z * p.A_q * p.n_bin * M;
    for (int al = 0; al < p.A_q; ++al) {
        const float* ya = yz + (size_t)al * p.n_bin * M;
        pixel_footprint(sA[al], xc, yc, p.n_bin, p.du, p.inv_du, [&](int b, float len) {
            float v[M];
            load_record<M>(ya + (size_t)b * M, v);
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] = fmaf(len, v[m], acc[m]);
            sens += len;
        });
    }
}

template <int M>
__host__ __device__ __forceinline__ void backproject_voxel(const AngleRec* sA, const ProjArgs& p,
                                                           const float* __restrict__ y, float* __restrict__ bout,
                                                           float* __restrict__ sens_out, int i, int j, int z) {
    float acc[M], sens;
    gather<M>(sA, p, y, i, j, z, acc, sens);
    const size_t v = ((size_t)z * p.ny + j) * p.nx + i;
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] *= p.fr.E[m];
    store_record<M>(bout + v * M, acc);
    if (sens_out) sens_out[v] = sens;
}

// OSL-KP update of voxel (i, j, z).  Fm: model TACs of the current maps [N][M] (only read when
// the prior is on).
template <int M>
__host__ __device__ __forceinline__ void osl_voxel(const AngleRec* sA, const OslArgs& a, const float* __restrict__ ratio,
                                                   const float* __restrict__ Fm, float* __restrict__ x, int i, int j,
                                                   int z) {
    const ProjArgs& p = a.g;
    float acc[M], sens;
    gather<M>(sA, p, ratio, i, j, z, acc, sens);
    if (!(sens > 0.0f)) return;  // no ray of this subset sees the voxel: keep x
    const size_t v = ((size_t)z * p.ny + j) * p.nx + i;
    float xv[M];
    load_record<M>(x + v * M, xv);
    const float inv_sens = 1.0f / sens;
    if (a.kp) {
        float F[M];
        load_record<M>(Fm + v * M, F);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float d = fmaf(a.beta_kp, (xv[m] - F[m]) / fmaxf(F[m], a.eps_F), 1.0f);
            xv[m] = xv[m] * acc[m] * inv_sens / d;
        }
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) xv[m] = xv[m] * acc[m] * inv_sens;
    }
    store_record<M>(x + v * M, xv);
}

template <int M, class Src>
__global__ __launch_bounds__(256) void kback_kernel(Src src) {
    extern __shared__ AngleRec sA[];
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const BackJob& J = src.find(w);
    subset_angles_to_lds(sA, J.p);
    const TileIdx t = tile_voxel(w - J.w0, J.p.nx, J.p.ny, J.p.nz);
    if (!t.valid) return;
    backproject_voxel<M>(sA, J.p, J.y, J.b, J.sens, t.i, t.j, t.z);
}

template <int M, class Src>
__global__ __launch_bounds__(256) void kosl_kernel(Src src) {
    extern __shared__ AngleRec sA[];
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const OslJob& J = src.find(w);
    subset_angles_to_lds(sA, J.a.g);
    const TileIdx t = tile_voxel(w - J.w0, J.a.g.nx, J.a.g.ny, J.a.g.nz);
    if (!t.valid) return;
    osl_voxel<M>(sA, J.a, J.ratio, J.Fm, J.x, t.i, t.j, t.z);
}

template <int M, class Src>
static hipError_t launch_back_m(Src src, uint32_t groups, int max_angles, hipStream_t st) {
    hipLaunchKernelGGL((kback_kernel<M, Src>), dim3(xcd_round_up(groups)), dim3(kTileX * kTileY),
                       max_angles * sizeof(AngleRec), st, src);
    return hipGetLastError();
}

template <int M, class Src>
static hipError_t launch_osl_m(Src src, uint32_t groups, int max_angles, hipStream_t st) {
    hipLaunchKernelGGL((kosl_kernel<M, Src>), dim3(xcd_round_up(groups)), dim3(kTileX * kTileY),
                       max_angles * sizeof(AngleRec), st, src);
    return hipGetLastError();
}

hipError_t launch_backproject(int M, const float* y, float* b, float* sens, const ProjArgs& p, hipStream_t st) {
    if (p.A_q > kMaxSubsetAngles) return hipErrorInvalidValue;
    OneJob<BackJob> src{BackJob{p, y, b, sens, 0}};
    const uint32_t g = voxel_tile_groups(p.nx, p.ny, p.nz);
    switch (M) {
        case 8: return launch_back_m<8>(src, g, p.A_q, st);
        case 16: return launch_back_m<16>(src, g, p.A_q, st);
        case 24: return launch_back_m<24>(src, g, p.A_q, st);
        case 32: return launch_back_m<32>(src, g, p.A_q, st);
        default: return hipErrorInvalidValue;
    }
}

template <class Src>
static hipError_t dispatch_osl(int M, Src src, uint32_t groups, int max_angles, hipStream_t st) {
    if (max_angles > kMaxSubsetAngles) return hipErrorInvalidValue;
    switch (M) {
        case 8: return launch_osl_m<8>(src, groups, max_angles, st);
        case 16: return launch_osl_m<16>(src, groups, max_angles, st);
        case 24: return launch_osl_m<24>(src, groups, max_angles, st);
        case 32: return launch_osl_m<32>(src, groups, max_angles, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_osl(int M, const float* ratio, const float* Fm, float* x, const OslArgs& a, hipStream_t st) {
    OneJob<OslJob> src{OslJob{a, ratio, Fm, x, 0}};
    return dispatch_osl(M, src, voxel_tile_groups(a.g.nx, a.g.ny, a.g.nz), a.g.A_q, st);
}

hipError_t launch_osl_jobs(int M, const OslJob* jobs, int n, uint32_t groups, int max_angles, hipStream_t st) {
    return dispatch_osl(M, JobTable<OslJob>{jobs, n}, groups, max_angles, st);
}

}  // namespace kcs
