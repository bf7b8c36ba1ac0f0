// K-proj: ray-driven forward projector (denominator of Eq. 2) with exact Siddon lengths.
//
// One thread per ray of the subset; the thread walks the pixels the ray crosses in order
// (incremental Siddon traversal in pixel units) and accumulates all M frames of each crossed
// pixel's record into registers, so each voxel record is read as M/4 16-byte loads and the
// traversal is shared by the frames.  Output rays of one (plane, angle) are contiguous and
// each thread writes its M-frame record, so the write stream is dense.
// In ratio mode the thread also forms ybar = E_m * sum + r_m and writes s / ybar (the
// measured-to-expected ratio that the OSL back projection consumes).
#include "kcs_device.h"
#include "kcs_launch.h"

namespace kcs {

// Ray (z, al, b) of subset p.q: ybar = E_m sum + r_m, or the ratio s / ybar.
template <int M, bool RATIO>
__host__ __device__ __forceinline__ void project_ray(const ProjArgs& p, const float* __restrict__ x,
                                                     const float* __restrict__ sino, float* __restrict__ out, int z,
                                                     int al, int b) {
    const int a = p.q + al * p.Q;  // global angle index
    const AngleRec A = make_angle(a, p.n_ang, p.ang0, p.h);
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

template <int M, bool RATIO>
__global__ __launch_bounds__(256) void kproj_kernel(const float* __restrict__ x, const float* __restrict__ sino,
                                                    float* __restrict__ out, ProjArgs p) {
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const uint32_t blocks_per_plane = (p.rays_per_plane + 255u) / 256u;
    const uint32_t z = w / blocks_per_plane;
    if (z >= (uint32_t)p.nz) return;
    const uint32_t ray = (w % blocks_per_plane) * 256u + threadIdx.x;
    if (ray >= (uint32_t)p.rays_per_plane) return;
    const int al = ray / p.n_bin;  // angle within the subset
    project_ray<M, RATIO>(p, x, sino, out, z, al, ray - al * p.n_bin);
}

template <int M>
static hipError_t launch_proj_m(const float* x, const float* sino, float* out, const ProjArgs& p, bool ratio,
                                hipStream_t st) {
    const uint32_t bpp = (p.rays_per_plane + 255u) / 256u;
    const uint32_t n = xcd_round_up(bpp * (uint32_t)p.nz);
    if (ratio)
        hipLaunchKernelGGL((kproj_kernel<M, true>), dim3(n), dim3(256), 0, st, x, sino, out, p);
    else
        hipLaunchKernelGGL((kproj_kernel<M, false>), dim3(n), dim3(256), 0, st, x, sino, out, p);
    return hipGetLastError();
}

hipError_t launch_project(int M, const float* x, const float* sino, float* out, const ProjArgs& p, bool ratio,
                          hipStream_t st) {
    switch (M) {
        case 8: return launch_proj_m<8>(x, sino, out, p, ratio, st);
        case 16: return launch_proj_m<16>(x, sino, out, p, ratio, st);
        case 24: return launch_proj_m<24>(x, sino, out, p, ratio, st);
        case 32: return launch_proj_m<32>(x, sino, out, p, ratio, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace kcs
