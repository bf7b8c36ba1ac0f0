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
uint32_t model_groups(int64_t n) { return (uint32_t)((n + 255) / 256); }

template <int M, bool JAC, class Src>
__global__ __launch_bounds__(256) void kmodel_kernel(Src src) {
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const ModelJob& Jb = src.find(w);
    const int64_t n = Jb.n;
    const int64_t v = (int64_t)(w - Jb.w0) * 256 + threadIdx.x;
    if (v >= n) return;
    const float* params = Jb.params;
    float f[M], jac[JAC ? 3 * M : 1];
    model_frames<M, JAC>(Jb.fr, *Jb.K, params[v], params[n + v], params[2 * n + v],
                         [&](int m, float Fm, float a, float b, float c) {
                             f[m] = Fm;
                             if (JAC) {
                                 jac[3 * m] = a;
                                 jac[3 * m + 1] = b;
                                 jac[3 * m + 2] = c;
                             }
                         });
    store_record<M>(Jb.F + v * M, f);
    if (JAC) {
#pragma unroll
        for (int k = 0; k < 3 * M; ++k) Jb.J[v * 3 * M + k] = jac[k];
    }
}

template <class Src>
static hipError_t dispatch_model(int M, bool jac, Src src, uint32_t groups, hipStream_t st) {
    const dim3 g(xcd_round_up(groups)), b(256);
#define KCS_MODEL_CASE(MM)                                                                   \
    case MM:                                                                                 \
        if (jac)                                                                             \
            hipLaunchKernelGGL((kmodel_kernel<MM, true, Src>), g, b, 0, st, src);            \
        else                                                                                 \
            hipLaunchKernelGGL((kmodel_kernel<MM, false, Src>), g, b, 0, st, src);           \
        break;
    switch (M) {
        KCS_MODEL_CASE(8)
        KCS_MODEL_CASE(16)
        KCS_MODEL_CASE(24)
        KCS_MODEL_CASE(32)
        default: return hipErrorInvalidValue;
    }
#undef KCS_MODEL_CASE
    return hipGetLastError();
}

hipError_t launch_model(int M, const KinTab* K, const FrameTab& fr, const float* params, int64_t n, float* F, float* J,
                        hipStream_t st) {
    OneJob<ModelJob> src{ModelJob{fr, K, params, n, F, J, 0}};
    return dispatch_model(M, J != nullptr, src, model_groups(n), st);
}

hipError_t launch_model_jobs(int M, JobTable<ModelJob> jobs, uint32_t groups, hipStream_t st) {
    return dispatch_model(M, false, jobs, groups, st);
}

// Net uptake rate K_i = K1 k3 / (k2 + k3) per voxel (the macro-parameter of Sec. IV); where
// k2 + k3 = 0 nothing leaves the first compartment and K_i = K1.  params [3][n], ki [n].
__global__ __launch_bounds__(256) void kki_kernel(const float* __restrict__ params, int64_t n,
                                                  float* __restrict__ ki) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float K1 = params[e], k2 = params[n + e], k3 = params[2 * n + e];
    const float a = k2 + k3;
    ki[e] = a > 0.0f ? K1 * k3 / a : K1;
}

hipError_t launch_ki(const float* params, int64_t n, float* ki, hipStream_t st) {
    const int64_t groups = (n + 255) / 256;
    hipLaunchKernelGGL(kki_kernel, dim3((uint32_t)groups), dim3(256), 0, st, params, n, ki);
    return hipGetLastError();
}

// Batched device-to-device copies (the kinetic maps before an odd number of LM iterations).
uint32_t copy_groups(int64_t n) { return (uint32_t)((n + 1023) / 1024); }

__global__ __launch_bounds__(256) void kcopy_kernel(JobTable<CopyJob> src) {
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const CopyJob& J = src.find(w);
    const int64_t base = (int64_t)(w - J.w0) * 1024 + threadIdx.x;
    for (int k = 0; k < 4; ++k) {
        const int64_t e = base + k * 256;
        if (e < J.n) J.dst[e] = J.src[e];
    }
}

hipError_t launch_copy_jobs(JobTable<CopyJob> jobs, uint32_t groups, hipStream_t st) {
    hipLaunchKernelGGL(kcopy_kernel, dim3(xcd_round_up(groups)), dim3(256), 0, st, jobs);
    return hipGetLastError();
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
