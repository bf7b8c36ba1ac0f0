// Streaming kernels for measurement harnesses: the HBM rate this GPU sustains for a plain read
// and a plain copy, the ceilings the bandwidth-bound kernels are compared with.
#include "kcs_device.h"
#include "kcs_launch.h"

namespace kcs {

constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 4;  // float4 loads in flight per thread and iteration

// Reads n4 float4s with a grid-stride loop and writes one partial sum per thread (so the loads
// cannot be dropped): out holds gridDim.x * blockDim.x floats.
__global__ __launch_bounds__(kStreamThreads) void kstream_read_kernel(const float4* __restrict__ src, size_t n4,
                                                                      float* __restrict__ out) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (; i + (kStreamUnroll - 1) * stride < n4; i += kStreamUnroll * stride) {
        float4 v[kStreamUnroll];
#pragma unroll
        for (int k = 0; k < kStreamUnroll; ++k) v[k] = src[i + k * stride];
#pragma unroll
        for (int k = 0; k < kStreamUnroll; ++k) {
            acc.x += v[k].x;
            acc.y += v[k].y;
            acc.z += v[k].z;
            acc.w += v[k].w;
        }
    }
    for (; i < n4; i += stride) {
        const float4 v = src[i];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc.x + acc.y + acc.z + acc.w;
}

__global__ __launch_bounds__(kStreamThreads) void kstream_copy_kernel(const float4* __restrict__ src, size_t n4,
                                                                      float4* __restrict__ dst) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kStreamUnroll - 1) * stride < n4; i += kStreamUnroll * stride) {
        float4 v[kStreamUnroll];
#pragma unroll
        for (int k = 0; k < kStreamUnroll; ++k) v[k] = src[i + k * stride];
#pragma unroll
        for (int k = 0; k < kStreamUnroll; ++k) dst[i + k * stride] = v[k];
    }
    for (; i < n4; i += stride) dst[i] = src[i];
}

size_t stream_read_out_floats(int groups) { return (size_t)groups * kStreamThreads; }

hipError_t launch_stream(int kind, const void* src, void* dst, size_t bytes, int groups, hipStream_t st) {
    const size_t n4 = bytes / 16;
    if (kind == 0)
        hipLaunchKernelGGL(kstream_read_kernel, dim3(groups), dim3(kStreamThreads), 0, st,
                           static_cast<const float4*>(src), n4, static_cast<float*>(dst));
    else
        hipLaunchKernelGGL(kstream_copy_kernel, dim3(groups), dim3(kStreamThreads), 0, st,
                           static_cast<const float4*>(src), n4, static_cast<float4*>(dst));
    return hipGetLastError();
}

}  // namespace kcs
