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

// F (and with JAC the Jacobian, [n][M][NP]) of n voxels whose maps are params [NP][n]: NP = 3
// (K1, k2, k3; the study's blood fraction) or 4 (plus the voxel's blood fraction vb).
template <int M, bool JAC, int NP, class Src>
__global__ __launch_bounds__(256) void kmodel_kernel(Src src) {
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const ModelJob& Jb = src.find(w);
    const int64_t n = Jb.n;
    const int64_t v = (int64_t)(w - Jb.w0) * 256 + threadIdx.x;
    if (v >= n) return;
    const float* params = Jb.params;
    float f[M], jac[JAC ? NP * M : 1];
    model_frames<M, JAC, true, NP>(Jb.fr, *Jb.K, params[v], params[n + v], params[2 * n + v],
                                   NP == 4 ? params[3 * n + v] : 0.0f,
                                   [&](int m, float Fm, float a, float b, float c, float d) {
                                       f[m] = Fm;
                                       if (JAC) {
                                           jac[NP * m] = a;
                                           jac[NP * m + 1] = b;
                                           jac[NP * m + 2] = c;
                                           if (NP == 4) jac[NP * m + 3] = d;
                                       }
                                   });
    store_record<M>(Jb.F + v * M, f);
    if (JAC) {
#pragma unroll
        for (int k = 0; k < NP * M; ++k) Jb.J[v * NP * M + k] = jac[k];
    }
}

template <int NP, class Src>
static hipError_t dispatch_model_np(int M, bool jac, Src src, uint32_t groups, hipStream_t st) {
    const dim3 g(xcd_round_up(groups)), b(256);
#define KCS_MODEL_CASE(MM)                                                                   \
    case MM:                                                                                 \
        if (jac)                                                                             \
            hipLaunchKernelGGL((kmodel_kernel<MM, true, NP, Src>), g, b, 0, st, src);        \
        else                                                                                 \
            hipLaunchKernelGGL((kmodel_kernel<MM, false, NP, Src>), g, b, 0, st, src);       \
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

template <class Src>
static hipError_t dispatch_model(int M, int np, bool jac, Src src, uint32_t groups, hipStream_t st) {
    if (np == 4) return dispatch_model_np<4>(M, jac, src, groups, st);
    if (np == 3) return dispatch_model_np<3>(M, jac, src, groups, st);
    return hipErrorInvalidValue;
}

hipError_t launch_model(int M, int np, const KinTab* K, const FrameTab& fr, const float* params, int64_t n, float* F,
                        float* J, hipStream_t st) {
    OneJob<ModelJob> src{ModelJob{fr, K, params, n, F, J, 0}};
    return dispatch_model(M, np, J != nullptr, src, model_groups(n), st);
}

hipError_t launch_model_jobs(int M, JobTable<ModelJob> jobs, uint32_t groups, hipStream_t st) {
    return dispatch_model(M, 3, false, jobs, groups, st);
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

// Initial maps: the np values of xi0 (K1, k2, k3 and, with np = 4, the blood fraction).
struct InitMaps {
    float v[4];
    int32_t np;
};

template <int M>
__global__ __launch_bounds__(256) void init_fill_kernel(const double* __restrict__ x0, int64_t N, InitMaps xi0,
                                                        float* __restrict__ x, float* __restrict__ params,
                                                        float* __restrict__ lam) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    float r[M];
#pragma unroll
    for (int m = 0; m < M; ++m) r[m] = (float)x0[m];
    store_record<M>(x + v * M, r);
    for (int k = 0; k < xi0.np; ++k) params[k * N + v] = xi0.v[k];
    lam[v] = 0.0f;
}

hipError_t launch_init(int M, const float* sino, int64_t rows, const FrameTab& fr, double denom_scale, int32_t N,
                       const double* xi0, int32_t np, double* partial, int32_t n_chunks, float* x, float* params,
                       float* lam, hipStream_t st) {
    const int64_t threads = (int64_t)n_chunks * M;
    hipLaunchKernelGGL(init_partial_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, st, sino, rows, M,
                       n_chunks, partial);
    double* x0 = partial + (int64_t)n_chunks * M;
    hipLaunchKernelGGL(init_frame_kernel, dim3(1), dim3(kMaxFrames), 0, st, partial, n_chunks, rows, fr, denom_scale, x0);
    const uint32_t blocks = (uint32_t)((N + 255) / 256);
    InitMaps im{};
    im.np = np;
    for (int k = 0; k < np; ++k) im.v[k] = (float)xi0[k];
    switch (M) {
        case 8: hipLaunchKernelGGL((init_fill_kernel<8>), dim3(blocks), dim3(256), 0, st, x0, (int64_t)N, im, x, params, lam); break;
        case 16: hipLaunchKernelGGL((init_fill_kernel<16>), dim3(blocks), dim3(256), 0, st, x0, (int64_t)N, im, x, params, lam); break;
        case 24: hipLaunchKernelGGL((init_fill_kernel<24>), dim3(blocks), dim3(256), 0, st, x0, (int64_t)N, im, x, params, lam); break;
        case 32: hipLaunchKernelGGL((init_fill_kernel<32>), dim3(blocks), dim3(256), 0, st, x0, (int64_t)N, im, x, params, lam); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace kcs
