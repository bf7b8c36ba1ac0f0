// Kernel launchers and their argument blocks (host side of libkcs).
#pragma once

#include "kcs_internal.h"

namespace kcs {

// Arguments common to the projector kernels (passed by value).
struct ProjArgs {
    int32_t nx, ny, nz, n_ang, n_bin;
    int32_t q, Q, A_q;        // subset q of Q holds angles q, q+Q, ...; A_q of them
    int32_t rays_per_plane;   // A_q * n_bin
    float h, inv_h, du, inv_du;
    double ang0;
    double hd, dud;  // pixel side and bin width in FP64 (ray positions relative to tiles)
    const float* mult;  // [nz][n_ang][n_bin] multiplicative correction per ray, or NULL (ones)
    FrameTab fr;
};

// Arguments of the OSL update: projector geometry plus the prior.
struct OslArgs {
    ProjArgs g;
    float beta_kp, eps_F;
    int32_t kp;
};

// Arguments of one MAP-LM iteration.
struct LmArgs {
    int32_t nx, ny, nz;
    FrameTab fr;
    float beta_h;
    int32_t np;  // fitted parameters: 3 (K1, k2, k3) or 4 (and the blood fraction vb)
    float delta[4];
    // 3x3x3 neighbourhood when nbr3d: weights of the through-plane neighbours with 0, 1 or 2
    // in-plane offsets (1 / distance in pixel sides)
    int32_t nbr3d;
    float w_plane[3];
    float tau, lam_min, lam_max;
    float eta;  // sufficient relative decrease of the objective for accepting a step
    int32_t reset_lambda;  // 1: ignore the stored lambda and start from tau * max diag(J^T J)
    // Normal-equation state carried between the iterations of one fit (see klm_kernel):
    int32_t have_state;    // 1: J^T J, J^T r and r^T r at the current maps are in `state`
    int32_t need_state;    // 1: leave them in `state` for the next iteration
    float lo[4], hi[4];
    int32_t tile_x;  // voxel rows of tile_x voxels, 256 / tile_x of them per workgroup (see lm_tile_x)
};

// Inputs of the FP64 table-setup kernel.
struct SetupArgs {
    double A1, A2, A3, l[3], vb;
    int32_t n_bound;
    double t[kMaxBoundaries];
    int32_t M;
    int32_t i0[kMaxFrames], i1[kMaxFrames];
};

// ---------------------------------------------------------------------------------------------
// Jobs.  Every kernel processes a list of jobs (one per study); its workgroups are numbered over
// the concatenated work lists (after the XCD remap) and each finds its job by the first work
// index w0.  A single-study call passes one job by value; a batched plan passes a device table.
struct ProjJob {
    ProjArgs p;
    const float* x;
    const float* sino;
    float* out;
    float* psum;
    int32_t slots;
    uint32_t w0;
};
struct OslJob {
    OslArgs a;
    const float* ratio;
    const float* Fm;
    float* x;
    uint32_t w0;
};
struct BackJob {
    ProjArgs p;
    const float* y;
    float* b;
    float* sens;
    uint32_t w0;
};
struct LmJob {
    LmArgs a;
    const KinTab* K;
    const float* x;
    const float* xi_in;
    float* xi_out;
    float* lam;
    float* state;  // [10][N] (3 maps) or [15][N] (4): J^T J, J^T r, r^T r at the current maps
    uint32_t w0;
};
struct ModelJob {
    FrameTab fr;
    const KinTab* K;
    const float* params;
    int64_t n;
    float* F;
    float* J;
    uint32_t w0;
};
struct CopyJob {
    const float* src;
    float* dst;
    int64_t n;
    uint32_t w0;
};

template <class J>
struct OneJob {
    J job;
    __device__ __forceinline__ const J& find(uint32_t) const { return job; }
};

template <class J>
struct JobTable {
    const J* jobs;
    const uint32_t* starts;  // starts[k] = jobs[k].w0, ascending, packed for the search
    int32_t n;
    // The tables are read-only while a kernel runs, so they are read through the constant address
    // space: the job fields become scalar loads (the index is uniform per workgroup) and the
    // buffer pointers stored in the jobs are known to be global, which keeps the data accesses on
    // global (not flat) loads and stores.  The job is found by binary search over `starts`.
    __device__ __forceinline__ const J& find(uint32_t w) const {
        using CJ = const __attribute__((address_space(4))) J;
        using CU = const __attribute__((address_space(4))) uint32_t;
        CJ* t = (CJ*)jobs;
        CU* s = (CU*)starts;
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s[mid] <= w)
                lo = mid;
            else
                hi = mid - 1;
        }
        return *(const J*)&t[lo];
    }
};

// Workgroups each job needs.
uint32_t proj_direct_groups(const ProjArgs& p);
uint32_t proj_reduce_groups(const ProjArgs& p);
uint32_t proj_tile_groups(const ProjArgs& p, int T);
uint32_t staged_tile_groups(int nx, int ny, int nz);
bool staged_fits(int M, float h, float du);  // one angle's staged bin records fit in the LDS
int lm_tile_x(int nx, int ny);
uint32_t lm_groups(int nx, int ny, int nz, int tile_x);
uint32_t model_groups(int64_t n);
uint32_t copy_groups(int64_t n);

// Launchers over job tables (device tables of n jobs covering `groups` workgroups in total).
hipError_t launch_project_jobs(int M, int T, JobTable<ProjJob> jobs, uint32_t groups, int max_angles, bool ratio,
                               hipStream_t st);
hipError_t launch_project_reduce_jobs(int M, int T, JobTable<ProjJob> jobs, uint32_t groups, bool ratio,
                                      hipStream_t st);
hipError_t launch_osl_jobs(int M, JobTable<OslJob> jobs, uint32_t groups, int max_angles, hipStream_t st);
hipError_t launch_lm_jobs(int M, bool nbr3d, JobTable<LmJob> jobs, uint32_t groups, hipStream_t st);
hipError_t launch_model_jobs(int M, JobTable<ModelJob> jobs, uint32_t groups, hipStream_t st);
hipError_t launch_copy_jobs(JobTable<CopyJob> jobs, uint32_t groups, hipStream_t st);

hipError_t launch_setup(const SetupArgs& s, KinTab* K, hipStream_t st);
hipError_t launch_project(int M, const float* x, const float* sino, float* out, const ProjArgs& p, bool ratio,
                          hipStream_t st);
hipError_t launch_project_tiled(int M, int T, const float* x, const float* sino, float* out, float* psum,
                                const ProjArgs& p, bool ratio, hipStream_t st);
size_t tile_partial_bytes(int T, const ProjArgs& p, int M);
hipError_t launch_backproject(int M, const float* y, float* b, float* sens, const ProjArgs& p, hipStream_t st);
hipError_t launch_osl(int M, const float* ratio, const float* Fm, float* x, const OslArgs& a, hipStream_t st);
hipError_t launch_lm(int M, const KinTab* K, const float* x, const float* xi_in, float* xi_out, float* lam,
                     float* state, const LmArgs& a, hipStream_t st);
hipError_t launch_ki(const float* params, int64_t n, float* ki, hipStream_t st);

// Single-slice rebinning: R rings, ring differences up to D, sinograms of n_ang x n_bin x M.
struct RebinArgs {
    int32_t R, D, n_ang, n_bin, M;
};
hipError_t launch_ssrb(const RebinArgs& a, const float* y3d, float* y2d, float* count, hipStream_t st);

// Streaming read (kind 0: one partial sum per thread into dst, stream_read_out_floats(groups)
// floats) or copy (kind 1) of bytes (a multiple of 16) for bandwidth measurement.
size_t stream_read_out_floats(int groups);
hipError_t launch_stream(int kind, const void* src, void* dst, size_t bytes, int groups, hipStream_t st);
hipError_t launch_model(int M, int np, const KinTab* K, const FrameTab& fr, const float* params, int64_t n, float* F,
                        float* J, hipStream_t st);
hipError_t launch_init(int M, const float* sino, int64_t rows, const FrameTab& fr, double denom_scale, int32_t nz_ny_nx,
                       const double* xi0, int32_t np, double* partial, int32_t n_chunks, float* x, float* params,
                       float* lam, hipStream_t st);

}  // namespace kcs
