// Single-slice rebinning (SSRB) of a span-1 3D acquisition into the 2R - 1 direct and cross
// planes that the direct-plane reconstruction takes (the 3D listmode data of Sec. IV, rebinned
// into sinograms).  The line of response between rings r1 and r2 has its axial midpoint on plane
// z = r1 + r2 of planes spaced half a ring apart; rebinning adds its sinogram into that plane.
// One thread per output value (plane, angle, bin, frame): consecutive threads read consecutive
// values of each input sinogram, so the input is streamed once, in order of ring difference.
#include "kcs_device.h"
#include "kcs_launch.h"

namespace kcs {

constexpr int kRebinThreads = 256;

// Number of ring pairs (r1, r2), |r2 - r1| <= D, 0 <= r1, r2 < R, with r1 + r2 = z.
__host__ __device__ inline int ssrb_pairs(int R, int D, int z) {
    int n = 0;
    for (int delta = -D; delta <= D; ++delta) {
        if (((z - delta) & 1) != 0) continue;
        const int r1 = (z - delta) / 2, r2 = r1 + delta;
        n += (r1 >= 0 && r1 < R && r2 >= 0 && r2 < R) ? 1 : 0;
    }
    return n;
}

__global__ __launch_bounds__(kRebinThreads) void kssrb_kernel(RebinArgs a, const float* __restrict__ y3d,
                                                              float* __restrict__ y2d, float* __restrict__ count) {
    const int64_t per_plane = (int64_t)a.n_ang * a.n_bin * a.M;  // values of one sinogram
    const int64_t e = (int64_t)blockIdx.x * kRebinThreads + threadIdx.x;
    const int64_t total = (int64_t)(2 * a.R - 1) * per_plane;
    if (e >= total) return;
    const int z = (int)(e / per_plane);
    const int64_t off = e - (int64_t)z * per_plane;
    // the ring differences of plane z: delta = r2 - r1 with r1 + r2 = z, both rings in [0, R),
    // |delta| <= D and delta of the parity of z; summed in increasing order
    int lo = max(max(-a.D, -z), z - 2 * a.R + 2);
    const int hi = min(min(a.D, z), 2 * a.R - 2 - z);
    lo += (lo - z) & 1;
    float acc = 0.0f;
#pragma unroll 4
    for (int delta = lo; delta <= hi; delta += 2)
        acc += y3d[((int64_t)(delta + a.D) * a.R + (z - delta) / 2) * per_plane + off];
    y2d[e] = acc;
    if (count && off == 0) count[z] = (float)ssrb_pairs(a.R, a.D, z);
}

hipError_t launch_ssrb(const RebinArgs& a, const float* y3d, float* y2d, float* count, hipStream_t st) {
    const int64_t total = (int64_t)(2 * a.R - 1) * a.n_ang * a.n_bin * a.M;
    const int64_t groups = (total + kRebinThreads - 1) / kRebinThreads;
    hipLaunchKernelGGL(kssrb_kernel, dim3((uint32_t)groups), dim3(kRebinThreads), 0, st, a, y3d, y2d, count);
    return hipGetLastError();
}

}  // namespace kcs
