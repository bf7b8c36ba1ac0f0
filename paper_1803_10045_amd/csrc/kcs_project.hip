// K-proj: ray-driven forward projector (denominator of Eq. 2) with exact Siddon lengths.
//
// One thread per ray of the subset; the thread walks the pixels the ray crosses in order
// (incremental Siddon traversal in pixel units) and accumulates all M frames of each crossed
// pixel's record into registers, so each voxel record is read as M/4 16-byte loads and the
// traversal is shared by the frames.  Output rays of one (plane, angle) are contiguous and
// each thread writes its M-frame record, so the write stream is dense.
// In ratio mode the thread also forms ybar = E_m * sum + r_m and writes s / ybar (the
// measured-to-expected ratio that the OSL back projection consumes).
//
// Tiled variant (large images): the image of one plane does not fit in an XCD's L2, so the
// ray-driven kernel re-reads it once per angle.  kproj_tile_kernel instead stages one T x T
// tile (all M frames) in LDS per workgroup and traverses, inside the tile, every subset ray that
// can meet it, writing one partial line integral per (tile, ray).  kproj_reduce_kernel adds the
// partials of each ray over the tiles in a fixed order (deterministic, no atomics) and applies
// the same epilogue.  The image then crosses HBM once per subset.
//
// All kernels take a job source: one study by value, or a device table of studies.
#include "kcs_device.h"
#include "kcs_launch.h"

namespace kcs {

// Expected counts or measured/expected ratio of ray (z, al, b) from its line integrals acc.
template <int M, bool RATIO>
__host__ __device__ __forceinline__ void ray_epilogue(const ProjArgs& p, const float* __restrict__ sino,
                                                      float* __restrict__ out, int z, int al, int b,
                                                      const float (&acc)[M]) {
    const int a = p.q + al * p.Q;
    const size_t o = (((size_t)z * p.A_q + al) * p.n_bin + b) * M;
    float y[M];
    if (RATIO) {
        float s[M];
        load_record<M>(sino + (((size_t)z * p.n_ang + a) * p.n_bin + b) * M, s);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float yb = fmaf(p.fr.E[m], acc[m], p.fr.r[m]);
            y[m] = yb > 0.0f ? s[m] / yb : 0.0f;
        }
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) y[m] = fmaf(p.fr.E[m], acc[m], p.fr.r[m]);
    }
    store_record<M>(out + o, y);
}

// Ray (z, al, b) of subset p.q through the whole plane.
template <int M, bool RATIO>
__host__ __device__ __forceinline__ void project_ray(const ProjArgs& p, const float* __restrict__ x,
                                                     const float* __restrict__ sino, float* __restrict__ out, int z,
                                                     int al, int b) {
    const AngleRec A = make_angle(p.q + al * p.Q, p.n_ang, p.ang0, p.h);
    float acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0f;
    const float u = ((float)b - 0.5f * (float)(p.n_bin - 1)) * p.du;
    const float* plane = x + (size_t)z * p.nx * p.ny * M;
    siddon_traverse(A, u, p.nx, p.ny, p.h, p.inv_h, [&](int i, int j, float len) {
        float v[M];
        load_record<M>(plane + ((size_t)j * p.nx + i) * M, v);
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] = fmaf(len, v[m], acc[m]);
    });
    ray_epilogue<M, RATIO>(p, sino, out, z, al, b, acc);
}

uint32_t proj_direct_groups(const ProjArgs& p) { return (uint32_t)((p.rays_per_plane + 255) / 256) * p.nz; }

template <int M, bool RATIO, class Src>
__global__ __launch_bounds__(256) void kproj_kernel(Src src) {
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const ProjJob& J = src.find(w);
    const ProjArgs& p = J.p;
    const uint32_t lw = w - J.w0;
    const uint32_t blocks_per_plane = (p.rays_per_plane + 255u) / 256u;
    const uint32_t z = lw / blocks_per_plane;
    if (z >= (uint32_t)p.nz) return;
    const uint32_t ray = (lw % blocks_per_plane) * 256u + threadIdx.x;
    if (ray >= (uint32_t)p.rays_per_plane) return;
    const int al = ray / p.n_bin;  // angle within the subset
    project_ray<M, RATIO>(p, J.x, J.sino, J.out, z, al, ray - al * p.n_bin);
}

uint32_t proj_tile_groups(const ProjArgs& p, int T) {
    return (uint32_t)(((p.nx + T - 1) / T) * ((p.ny + T - 1) / T)) * p.nz;
}

size_t tile_partial_bytes(int T, const ProjArgs& p, int M) {
    const size_t ntx = (p.nx + T - 1) / T, nty = (p.ny + T - 1) / T;
    return (size_t)p.nz * ntx * nty * p.A_q * tile_slots(T, p.h, p.du) * M * sizeof(float);
}

template <int M, int T, class Src>
__global__ __launch_bounds__(256) void kproj_tile_kernel(Src src) {
    extern __shared__ float4 lds4[];
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const ProjJob& J = src.find(w);
    const ProjArgs& p = J.p;
    const int slots = J.slots;
    AngleRec* sA = reinterpret_cast<AngleRec*>(lds4 + T * T * M / 4);
    const int ntx = (p.nx + T - 1) / T, nty = (p.ny + T - 1) / T;
    const uint32_t lw = w - J.w0;
    const int z = lw / (ntx * nty);
    if (z >= p.nz) return;  // whole workgroup
    const int tr = lw % (ntx * nty), ty = tr / ntx, tx = tr % ntx;
    const int i0 = tx * T, j0 = ty * T, tw = min(T, p.nx - i0), th = min(T, p.ny - j0);
    // stage the tile: row r of the tile is tw * M contiguous floats of the image
    const int row4 = tw * M / 4;
    const float4* src4 = reinterpret_cast<const float4*>(J.x) + (((size_t)z * p.ny + j0) * p.nx + i0) * (M / 4);
    for (int e = threadIdx.x; e < th * row4; e += blockDim.x) {
        const int r = e / row4, c = e - r * row4;
        lds4[r * (T * M / 4) + c] = src4[(size_t)r * p.nx * (M / 4) + c];
    }
    for (int al = threadIdx.x; al < p.A_q; al += blockDim.x) sA[al] = make_angle(p.q + al * p.Q, p.n_ang, p.ang0, p.h);
    __syncthreads();
    const float bc = 0.5f * (float)(p.n_bin - 1);
    const float* tile = reinterpret_cast<const float*>(lds4);
    float* out = J.psum + (((size_t)z * nty + ty) * ntx + tx) * (size_t)p.A_q * slots * M;
    for (int it = threadIdx.x; it < p.A_q * slots; it += blockDim.x) {
        const int al = it / slots, slot = it - al * slots;
        const AngleRec A = sA[al];
        int b0, b1;
        box_bins(A, i0, j0, tw, th, p.nx, p.ny, p.h, p.inv_du, p.n_bin, b0, b1);
        const int b = b0 + slot;
        if (b > b1) continue;
        float acc[M];
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] = 0.0f;
        const float u = ((float)b - bc) * p.du;
        const float Xc = u * A.c * p.inv_h + 0.5f * (float)p.nx - (float)i0;
        const float Yc = u * A.s * p.inv_h + 0.5f * (float)p.ny - (float)j0;
        siddon_traverse_box(A, Xc, Yc, tw, th, p.h, [&](int i, int j, float len) {
            float v[M];
            load_record<M>(tile + (j * T + i) * M, v);
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] = fmaf(len, v[m], acc[m]);
        });
        store_record<M>(out + (size_t)it * M, acc);
    }
}

template <int M, int T, bool RATIO, class Src>
__global__ __launch_bounds__(256) void kproj_reduce_kernel(Src src) {
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const ProjJob& J = src.find(w);
    const ProjArgs& p = J.p;
    const int slots = J.slots;
    const uint32_t lw = w - J.w0;
    const uint32_t blocks_per_plane = (p.rays_per_plane + 255u) / 256u;
    const uint32_t z = lw / blocks_per_plane;
    if (z >= (uint32_t)p.nz) return;
    const uint32_t ray = (lw % blocks_per_plane) * 256u + threadIdx.x;
    if (ray >= (uint32_t)p.rays_per_plane) return;
    const int al = ray / p.n_bin;
    const int b = ray - al * p.n_bin;
    const AngleRec A = make_angle(p.q + al * p.Q, p.n_ang, p.ang0, p.h);
    const int ntx = (p.nx + T - 1) / T, nty = (p.ny + T - 1) / T;
    float acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0f;
    const float* pz = J.psum + (size_t)z * nty * ntx * p.A_q * slots * M;
    for (int ty = 0; ty < nty; ++ty) {
        for (int tx = 0; tx < ntx; ++tx) {
            const int i0 = tx * T, j0 = ty * T;
            int b0, b1;
            box_bins(A, i0, j0, min(T, p.nx - i0), min(T, p.ny - j0), p.nx, p.ny, p.h, p.inv_du, p.n_bin, b0, b1);
            if (b < b0 || b > b1 || b - b0 >= slots) continue;
            float v[M];
            load_record<M>(pz + (((size_t)(ty * ntx + tx) * p.A_q + al) * slots + (b - b0)) * M, v);
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] += v[m];
        }
    }
    ray_epilogue<M, RATIO>(p, J.sino, J.out, z, al, b, acc);
}

// ---------------------------------------------------------------------------------------------
// Launch helpers

template <int M, int T, class Src>
static hipError_t launch_tile(Src src, uint32_t groups, int max_angles, hipStream_t st) {
    static bool attr_set = false;  // the tile may exceed the default 64 KB of dynamic LDS
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&kproj_tile_kernel<M, T, Src>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set = true;
    }
    const size_t lds = (size_t)T * T * M * sizeof(float) + (size_t)max_angles * sizeof(AngleRec);
    hipLaunchKernelGGL((kproj_tile_kernel<M, T, Src>), dim3(xcd_round_up(groups)), dim3(256), lds, st, src);
    return hipGetLastError();
}

template <int M, int T, class Src>
static hipError_t launch_reduce(Src src, uint32_t groups, bool ratio, hipStream_t st) {
    if (ratio)
        hipLaunchKernelGGL((kproj_reduce_kernel<M, T, true, Src>), dim3(xcd_round_up(groups)), dim3(256), 0, st, src);
    else
        hipLaunchKernelGGL((kproj_reduce_kernel<M, T, false, Src>), dim3(xcd_round_up(groups)), dim3(256), 0, st, src);
    return hipGetLastError();
}

template <int M, class Src>
static hipError_t launch_direct(Src src, uint32_t groups, bool ratio, hipStream_t st) {
    if (ratio)
        hipLaunchKernelGGL((kproj_kernel<M, true, Src>), dim3(xcd_round_up(groups)), dim3(256), 0, st, src);
    else
        hipLaunchKernelGGL((kproj_kernel<M, false, Src>), dim3(xcd_round_up(groups)), dim3(256), 0, st, src);
    return hipGetLastError();
}

// One step of the projector for frame count M and tile T (0 = ray-driven): the tile step
// (reduce_step = false) or the reduce step of a tiled projection, or the ray-driven kernel.
template <int M, class Src>
static hipError_t project_step(int T, Src src, uint32_t groups, int max_angles, bool ratio, bool reduce_step,
                               hipStream_t st) {
    if (T == 0) return reduce_step ? hipSuccess : launch_direct<M>(src, groups, ratio, st);
    if (T == 16)
        return reduce_step ? launch_reduce<M, 16>(src, groups, ratio, st) : launch_tile<M, 16>(src, groups, max_angles, st);
    if constexpr (M <= 24) {  // a 32 x 32 tile of 32 frames would exceed the LDS
        if (T == 32)
            return reduce_step ? launch_reduce<M, 32>(src, groups, ratio, st)
                               : launch_tile<M, 32>(src, groups, max_angles, st);
    }
    return hipErrorInvalidValue;
}

template <class Src>
static hipError_t dispatch_project(int M, int T, Src src, uint32_t groups, int max_angles, bool ratio,
                                   bool reduce_step, hipStream_t st) {
    switch (M) {
        case 8: return project_step<8>(T, src, groups, max_angles, ratio, reduce_step, st);
        case 16: return project_step<16>(T, src, groups, max_angles, ratio, reduce_step, st);
        case 24: return project_step<24>(T, src, groups, max_angles, ratio, reduce_step, st);
        case 32: return project_step<32>(T, src, groups, max_angles, ratio, reduce_step, st);
        default: return hipErrorInvalidValue;
    }
}

// Single study: ray-driven, or tiled with the partial buffer psum.
hipError_t launch_project(int M, const float* x, const float* sino, float* out, const ProjArgs& p, bool ratio,
                          hipStream_t st) {
    OneJob<ProjJob> src{ProjJob{p, x, sino, out, nullptr, 0, 0}};
    return dispatch_project(M, 0, src, proj_direct_groups(p), p.A_q, ratio, false, st);
}

hipError_t launch_project_tiled(int M, int T, const float* x, const float* sino, float* out, float* psum,
                                const ProjArgs& p, bool ratio, hipStream_t st) {
    if (T != 16 && T != 32) return hipErrorInvalidValue;
    OneJob<ProjJob> src{ProjJob{p, x, sino, out, psum, tile_slots(T, p.h, p.du), 0}};
    hipError_t e = dispatch_project(M, T, src, proj_tile_groups(p, T), p.A_q, ratio, false, st);
    if (e != hipSuccess) return e;
    return dispatch_project(M, T, src, proj_direct_groups(p), p.A_q, ratio, true, st);
}

// Batched: a device table of jobs.  For T > 0 the tile step and the reduce step are separate
// launches with separate tables (their work lists differ); max_angles bounds A_q over the jobs.
hipError_t launch_project_jobs(int M, int T, JobTable<ProjJob> jobs, uint32_t groups, int max_angles, bool ratio,
                               hipStream_t st) {
    return dispatch_project(M, T, jobs, groups, max_angles, ratio, false, st);
}

hipError_t launch_project_reduce_jobs(int M, int T, JobTable<ProjJob> jobs, uint32_t groups, bool ratio,
                                      hipStream_t st) {
    return dispatch_project(M, T, jobs, groups, 0, ratio, true, st);
}

}  // namespace kcs
