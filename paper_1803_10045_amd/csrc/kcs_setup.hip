// Table setup, model evaluation and initial-state kernels of libkcs.
//
// Setup: one small FP64 kernel turns the input-function parameters and the frame boundaries
// into the per-boundary constants of the closed-form tissue integral (KinTab), directly in the
// caller's workspace, so no host-to-device copy is needed and the calls stay asynchronous.
#include "kcs_device.h"
#include "kcs_launch.h"
#include "kcs_model.h"

namespace kcs {

__global__ void ktab_setup_kernel(SetupArgs s, KinTab* __restrict__ K) {
    const int b = threadIdx.x;
    if (b == 0) {
        for (int i = 0; i < kRates; ++i) K->l[i] = (float)s.l[i];
        K->w[0] = (float)s.A1;
        K->w[1] = (float)(-(s.A2 + s.A3));
        K->w[2] = (float)s.A2;
        K->w[3] = (float)s.A3;
        K->n_bound = s.n_bound;
        for (int m = 0; m < kMaxFrames; ++m) {
            K->i0[m] = m < s.M ? s.i0[m] : 0;
            K->i1[m] = m < s.M ? s.i1[m] : 0;
        }
    }
    if (b >= s.n_bound) return;
    K->b[b] = make_boundary(s.t[b], s.l);
}

hipError_t launch_setup(const SetupArgs& s, KinTab* K, hipStream_t st) {
    hipLaunchKernelGGL(ktab_setup_kernel, dim3(1), dim3(kMaxBoundaries), 0, st, s, K);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
template <int M, bool JAC>
__global__ __launch_bounds__(256) void kmodel_kernel(const KinTab* __restrict__ K, FrameTab fr,
                                                     const float* __restrict__ params, int64_t n, float* __restrict__ F,
                                                     float* __restrict__ J) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    float f[M], jac[3 * M];
    model_frames<M, JAC>(fr, *K, params[v], params[n + v], params[2 * n + v], [&](int m, float Fm, float a, float b, float c) {
        f[m] = Fm;
        if (JAC) {
            jac[3 * m] = a;
            jac[3 * m + 1] = b;
            jac[3 * m + 2] = c;
        }
    });
    store_record<M>(F + v * M, f);
    if (JAC) {
#pragma unroll
        for (int k = 0; k < 3 * M; ++k) J[v * 3 * M + k] = jac[k];
    }
}

template <int M>
static hipError_t launch_model_m(const KinTab* K, const FrameTab& fr, const float* params, int64_t n, float* F, float* J,
                                 hipStream_t st) {
    const uint32_t blocks = (uint32_t)((n + 255) / 256);
    if (J)
        hipLaunchKernelGGL((kmodel_kernel<M, true>), dim3(blocks), dim3(256), 0, st, K, fr, params, n, F, J);
    else
        hipLaunchKernelGGL((kmodel_kernel<M, false>), dim3(blocks), dim3(256), 0, st, K, fr, params, n, F, J);
    return hipGetLastError();
}

hipError_t launch_model(int M, const KinTab* K, const FrameTab& fr, const float* params, int64_t n, float* F, float* J,
                        hipStream_t st) {
    switch (M) {
        case 8: return launch_model_m<8>(K, fr, params, n, F, J, st);
        case 16: return launch_model_m<16>(K, fr, params, n, F, J, st);
        case 24: return launch_model_m<24>(K, fr, params, n, F, J, st);
        case 32: return launch_model_m<32>(K, fr, params, n, F, J, st);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------------------------
// Initial state.  Per-frame sinogram totals are reduced in FP64 in a fixed order (chunk c of
// rows by thread (c, m), then the chunks in order), so the result does not depend on timing.
__global__ void init_partial_kernel(const float* __restrict__ sino, int64_t rows, int32_t M, int32_t n_chunks,
                                    double* __restrict__ partial) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_chunks * M) return;
    const int32_t m = (int32_t)(t % M);
    const int64_t c = t / M;
    const int64_t per = (rows + n_chunks - 1) / n_chunks;
    const int64_t r0 = c * per, r1 = min(rows, r0 + per);
    double acc = 0.0;
    for (int64_t r = r0; r < r1; ++r) acc += (double)sino[r * M + m];
    partial[c * M + m] = acc;
}

__global__ void init_frame_kernel(const double* __restrict__ partial, int32_t n_chunks, int64_t rows, FrameTab fr,
                                  double denom_scale, double* __restrict__ x0) {
    const int m = threadIdx.x;
    if (m >= fr.M) return;
    double acc = 0.0;
    for (int c = 0; c < n_chunks; ++c) acc += partial[(int64_t)c * fr.M + m];
    const double net = acc - (double)fr.r[m] * (double)rows;
    x0[m] = fmax(net, 1.0) / ((double)fr.E[m] * denom_scale);
}

template <int M>
__global__ __launch_bounds__(256) void init_fill_kernel(const double* __restrict__ x0, int64_t N, double xi0_0,
                                                        double xi0_1, double xi0_2, float* __restrict__ x,
                                                        float* __restrict__ params, float* __restrict__ lam) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    float r[M];
#pragma unroll
    for (int m = 0; m < M; ++m) r[m] = (float)x0[m];
    store_record<M>(x + v * M, r);
    params[v] = (float)xi0_0;
    params[N + v] = (float)xi0_1;
    params[2 * N + v] = (float)xi0_2;
    lam[v] = 0.0f;
}

hipError_t launch_init(int M, const float* sino, int64_t rows, const FrameTab& fr, double denom_scale, int32_t N,
                       const double xi0[3], double* partial, int32_t n_chunks, float* x, float* params, float* lam,
                       hipStream_t st) {
    const int64_t threads = (int64_t)n_chunks * M;
    hipLaunchKernelGGL(init_partial_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, st, sino, rows, M,
                       n_chunks, partial);
    double* x0 = partial + (int64_t)n_chunks * M;
    hipLaunchKernelGGL(init_frame_kernel, dim3(1), dim3(kMaxFrames), 0, st, partial, n_chunks, rows, fr, denom_scale, x0);
    const uint32_t blocks = (uint32_t)((N + 255) / 256);
    switch (M) {
        case 8: hipLaunchKernelGGL((init_fill_kernel<8>), dim3(blocks), dim3(256), 0, st, x0, (int64_t)N, xi0[0], xi0[1], xi0[2], x, params, lam); break;
        case 16: hipLaunchKernelGGL((init_fill_kernel<16>), dim3(blocks), dim3(256), 0, st, x0, (int64_t)N, xi0[0], xi0[1], xi0[2], x, params, lam); break;
        case 24: hipLaunchKernelGGL((init_fill_kernel<24>), dim3(blocks), dim3(256), 0, st, x0, (int64_t)N, xi0[0], xi0[1], xi0[2], x, params, lam); break;
        case 32: hipLaunchKernelGGL((init_fill_kernel<32>), dim3(blocks), dim3(256), 0, st, x0, (int64_t)N, xi0[0], xi0[1], xi0[2], x, params, lam); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace kcs
