// K-back: voxel-driven (gather) back projector and the fused OS-MAP-OSL-KP update.
//
// One thread per voxel.  For each angle of the subset the voxel's footprint on the detector
// covers at most ceil(2 w1 / du) + 1 bins; the exact intersection length of each bin's ray with
// the voxel square (the pixel chord, identical to the Siddon length of that ray in that pixel)
// weights the bin's M-frame record.  The gather needs no atomics and no transposed system
// matrix.  A workgroup covers a 16 x 16 voxel tile, one voxel per thread: for a chunk of the
// subset's angles it stages in LDS the records of every bin whose ray can meet the tile, then
// each thread gathers its voxel's footprint from LDS.  The OSL update streams the image and the
// model TACs through HBM at about the device's copy rate; their loads are issued before the
// gather so that the latency hides behind it.
//
// OSL update (Eq. 2 with the kinetics-derived potential of Eq. 3, sigma^2 = F / n):
//   x_new = x * b / D,  b = E_m sum_d p_vd q_dm,  D = n_m (1 + beta (x - F) / max(F, eps_F)),
//   n_m = E_m sum_d p_vd;  E_m cancels between b and D.  x is kept where sum_d p_vd = 0.
// F, the model TAC of the current kinetic maps, does not change during an OSL pass; it is
// evaluated once per pass (kcs_model pass) and read here.
#include "kcs_device.h"
#include "kcs_launch.h"

namespace kcs {

constexpr int kMaxSubsetAngles = 1024;

// Per angle, the bins [b0, b1] whose rays can meet a pixel box and the signed distance tb from
// the centre of the box's corner pixel to ray b0, along the detector (mm).
struct BinRange {
    int32_t b0, b1;
    float tb, pad;
};

// The same, plus the bin range of every angle for the pixel box (i0, j0, tw, th).  tb is formed
// in FP64, so that a voxel's distance to a ray, tb + (b - b0) du - (its offset from the corner
// pixel projected on the detector), is a sum of terms no larger than the box: its FP32 error is
// that of the box's size, not of the distance to the image centre.
__device__ __forceinline__ void subset_angles_bins_to_lds(AngleRec* sA, BinRange* sBB, const ProjArgs& p, int i0,
                                                          int j0, int tw, int th) {
    for (int al = threadIdx.x; al < p.A_q; al += blockDim.x) {
        double c, s;
        angle_cos_sin(p.q + al * p.Q, p.n_ang, p.ang0, c, s);
        const AngleRec A = make_angle_cs(c, s, p.h);
        sA[al] = A;
        BinRange r;
        box_bins(A, i0, j0, tw, th, p.nx, p.ny, p.h, p.inv_du, p.n_bin, r.b0, r.b1);
        const double xc0 = ((double)i0 - 0.5 * (double)(p.nx - 1)) * p.hd;
        const double yc0 = ((double)j0 - 0.5 * (double)(p.ny - 1)) * p.hd;
        r.tb = (float)(((double)r.b0 - 0.5 * (double)(p.n_bin - 1)) * p.dud - (xc0 * c + yc0 * s));
        r.pad = 0.0f;
        sBB[al] = r;
    }
    __syncthreads();
}

// Loads voxel v's TAC (xv) and, when the prior is on, its model TAC from Fm [N][M] (F).  The
// update kernels issue these loads before their gather, so that the HBM latency is hidden
// behind it.
template <int M>
__host__ __device__ __forceinline__ void osl_load(const OslArgs& a, const float* __restrict__ Fm,
                                                  const float* __restrict__ x, size_t v, float (&xv)[M],
                                                  float (&F)[M]) {
    load_record<M>(x + v * M, xv);
    if (a.kp) load_record<M>(Fm + v * M, F);
}

// OSL-KP update of voxel v from its gathered acc, sens and the loaded xv, F; writes x.
template <int M>
__host__ __device__ __forceinline__ void osl_finish(const OslArgs& a, float* __restrict__ x, size_t v,
                                                    float (&xv)[M], const float (&F)[M], const float (&acc)[M],
                                                    float sens) {
    if (!(sens > 0.0f)) return;  // no ray of this subset sees the voxel: keep x
    const float inv_sens = 1.0f / sens;
    if (a.kp) {
        // x b / (n (1 + beta (x - F) / Fe)) = x (acc / sens) Fe / (Fe + beta (x - F)),  Fe = max(F, eps_F);
        // the denominator is at least (1 - beta) Fe > 0, so one hardware reciprocal (1 ulp) serves
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float fe = fmaxf(F[m], a.eps_F);
            const float den = fmaf(a.beta_kp, xv[m] - F[m], fe);
            xv[m] = xv[m] * acc[m] * inv_sens * fe * recip(den);
        }
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) xv[m] = xv[m] * acc[m] * inv_sens;
    }
    store_record<M>(x + v * M, xv);
}

constexpr int kST = 16;                // staged voxel tile: kST x kST voxels, one per thread
constexpr int kStageBytes = 20 * 1024;  // LDS for the staged bin records of one angle chunk

// Bins whose rays can meet a w x hgt pixel box: the box's projection is at most
// h sqrt(w^2 + hgt^2) wide, and box_bins widens it by a hundredth of a bin on each side.
__host__ __device__ inline int box_slots(int w, int hgt, float h, float du) {
    return (int)floorf(sqrtf((float)(w * w + hgt * hgt)) * h / du) + 3;
}

// LDS stride of a staged bin record in floats: padded by 4 (the first padding float holds the
// ray's correction factor) so that the records of nearby bins,
// which the voxels of a wavefront read at the same time, spread over the banks.
__host__ __device__ constexpr int stage_record(int M) { return M + 4; }

bool staged_fits(int M, float h, float du) {
    return box_slots(kST, kST, h, du) * stage_record(M) * (int)sizeof(float) <= kStageBytes;
}

uint32_t staged_tile_groups(int nx, int ny, int nz) {
    return (uint32_t)(((nx + kST - 1) / kST) * ((ny + kST - 1) / kST)) * nz;
}

// Angles per staging chunk for this geometry.
__host__ __device__ inline int stage_chunk(int M, int slots, int A_q) {
    const int c = kStageBytes / (slots * stage_record(M) * (int)sizeof(float));
    return max(1, min(c, A_q));
}

// For the voxel (i, j) of this thread in the staged tile (i0, j0) of plane z (valid: inside the
// image): acc_m = sum_{d in S_q} mu_d p_vd y_dm and sens = sum_{d in S_q} mu_d p_vd.  The staged
// record of bin d holds mu_d y_d and, in its first padding float, mu_d (1 without a correction
// sinogram).  All threads of the workgroup must call it (it synchronises).
template <int M>
__device__ __forceinline__ void staged_gather(const AngleRec* sA, const BinRange* sBB, float4* sR, const ProjArgs& p,
                                              const float* __restrict__ y, int z, bool valid, int i, int j, int i0,
                                              int j0, float (&acc)[M], float& sens) {
    const int slots = box_slots(kST, kST, p.h, p.du);
    const int chunk = stage_chunk(M, slots, p.A_q);
    // the voxel's centre relative to the centre of the tile's corner pixel (exact small multiples)
    const float dxc = (float)(i - i0) * p.h;
    const float dyc = (float)(j - j0) * p.h;
    sens = 0.0f;
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0f;
    const float4* yz = reinterpret_cast<const float4*>(y) + (size_t)z * p.A_q * p.n_bin * (M / 4);
    for (int c0 = 0; c0 < p.A_q; c0 += chunk) {
        const int na = min(chunk, p.A_q - c0);
        __syncthreads();  // previous chunk consumed
        for (int rec = threadIdx.x; rec < na * slots; rec += blockDim.x) {
            const int ar = rec / slots, al = c0 + ar, slot = rec - ar * slots;
            const BinRange bb = sBB[al];
            const int b = bb.b0 + slot;
            if (b > bb.b1) continue;
            const float4* src = yz + ((size_t)al * p.n_bin + b) * (M / 4);
            float4* dst = sR + rec * (stage_record(M) / 4);
            if (p.mult) {
                const float mu = p.mult[((size_t)z * p.n_ang + p.q + al * p.Q) * p.n_bin + b];
#pragma unroll
                for (int k = 0; k < M / 4; ++k) {
                    const float4 v = src[k];
                    dst[k] = make_float4(mu * v.x, mu * v.y, mu * v.z, mu * v.w);
                }
                dst[M / 4] = make_float4(mu, 0.0f, 0.0f, 0.0f);
            } else {
#pragma unroll
                for (int k = 0; k < M / 4; ++k) dst[k] = src[k];
                dst[M / 4] = make_float4(1.0f, 0.0f, 0.0f, 0.0f);
            }
        }
        __syncthreads();
        if (!valid) continue;
        for (int ac = 0; ac < na; ++ac) {
            const int al = c0 + ac;
            const AngleRec A = sA[al];
            const BinRange bb = sBB[al];
            // the voxel's footprint as in pixel_footprint, clipped to the staged bins [b0, b1]
            // (they hold every bin whose ray meets the tile, so the clip removes no chord); the
            // distance from the voxel centre to ray b is t = t0 + (b - b0) du
            const float t0 = bb.tb - fmaf(dxc, A.c, dyc * A.s);
            const float beta = -t0 * p.inv_du;  // the voxel centre in bins from b0
            const float rb = A.w1 * p.inv_du;
            const int lo = bb.b0 + max((int)ceilf(beta - rb), 0);
            const int hi = min(bb.b0 + (int)floorf(beta + rb), bb.b1);
            const float* rec = reinterpret_cast<const float*>(sR) + ((size_t)ac * slots + (lo - bb.b0)) * stage_record(M);
            float fk = (float)(lo - bb.b0);
            // every lane holds the same angle, so the chord form is a uniform branch
            const bool oblique = __builtin_amdgcn_readfirstlane(A.axis) == 0;
            for (int b = lo; b <= hi; ++b, fk += 1.0f, rec += stage_record(M)) {
                const float t = fmaf(fk, p.du, t0);
                const float len = oblique ? chord_oblique(A, t) : chord_axis(A, t);
                float v[M];
                load_record<M>(rec, v);
#pragma unroll
                for (int m = 0; m < M; ++m) acc[m] = fmaf(len, v[m], acc[m]);
                sens = fmaf(len, rec[M], sens);
            }
        }
    }
}

struct StagedTile {
    int i0, j0, z, i, j;
    bool valid;  // the thread's voxel (i, j) lies inside the image
};

__device__ __forceinline__ StagedTile staged_tile(uint32_t w, int nx, int ny, int nz) {
    const int ntx = (nx + kST - 1) / kST, nty = (ny + kST - 1) / kST;
    StagedTile t;
    t.z = w / (ntx * nty);
    const int r = w % (ntx * nty);
    t.j0 = (r / ntx) * kST;
    t.i0 = (r % ntx) * kST;
    t.i = t.i0 + (int)(threadIdx.x % kST);
    t.j = t.j0 + (int)(threadIdx.x / kST);
    t.valid = t.z < nz && t.i < nx && t.j < ny;
    return t;
}

template <int M, class Src>
__global__ __launch_bounds__(256) void kback_kernel(Src src) {
    extern __shared__ float4 lds[];
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const BackJob& J = src.find(w);
    const ProjArgs& p = J.p;
    const StagedTile t = staged_tile(w - J.w0, p.nx, p.ny, p.nz);
    if (t.z >= p.nz) return;  // whole workgroup
    AngleRec* sA = reinterpret_cast<AngleRec*>(lds);
    BinRange* sBB = reinterpret_cast<BinRange*>(lds + (p.A_q * sizeof(AngleRec) + 15) / 16);
    float4* sR = lds + (p.A_q * sizeof(AngleRec) + 15) / 16 + (p.A_q * sizeof(BinRange) + 15) / 16;
    subset_angles_bins_to_lds(sA, sBB, p, t.i0, t.j0, min(kST, p.nx - t.i0), min(kST, p.ny - t.j0));
    float acc[M], sens;
    staged_gather<M>(sA, sBB, sR, p, J.y, t.z, t.valid, t.i, t.j, t.i0, t.j0, acc, sens);
    if (!t.valid) return;
    const size_t v = ((size_t)t.z * p.ny + t.j) * p.nx + t.i;
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] *= p.fr.E[m];
    store_record<M>(J.b + v * M, acc);
    if (J.sens) J.sens[v] = sens;
}

template <int M, class Src>
__global__ __launch_bounds__(256) void kosl_kernel(Src src) {
    extern __shared__ float4 lds[];
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const OslJob& J = src.find(w);
    const OslArgs& a = J.a;
    const ProjArgs& p = a.g;
    const StagedTile t = staged_tile(w - J.w0, p.nx, p.ny, p.nz);
    if (t.z >= p.nz) return;  // whole workgroup
    AngleRec* sA = reinterpret_cast<AngleRec*>(lds);
    BinRange* sBB = reinterpret_cast<BinRange*>(lds + (p.A_q * sizeof(AngleRec) + 15) / 16);
    float4* sR = lds + (p.A_q * sizeof(AngleRec) + 15) / 16 + (p.A_q * sizeof(BinRange) + 15) / 16;
    subset_angles_bins_to_lds(sA, sBB, p, t.i0, t.j0, min(kST, p.nx - t.i0), min(kST, p.ny - t.j0));
    const size_t v = ((size_t)t.z * p.ny + t.j) * p.nx + t.i;
    float acc[M], sens, xv[M], F[M];
    if (t.valid) osl_load<M>(a, J.Fm, J.x, v, xv, F);
    staged_gather<M>(sA, sBB, sR, p, J.ratio, t.z, t.valid, t.i, t.j, t.i0, t.j0, acc, sens);
    if (t.valid) osl_finish<M>(a, J.x, v, xv, F, acc, sens);
}

static size_t staged_lds_bytes(int max_angles) {
    return (max_angles * sizeof(AngleRec) + 15) / 16 * 16 + (max_angles * sizeof(BinRange) + 15) / 16 * 16 +
           kStageBytes;
}

template <class K>
static void allow_large_lds(K kernel) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
}

template <int M, class Src>
static hipError_t launch_back_m(Src src, uint32_t groups, int max_angles, hipStream_t st) {
    static bool once = (allow_large_lds(&kback_kernel<M, Src>), true);
    (void)once;
    hipLaunchKernelGGL((kback_kernel<M, Src>), dim3(xcd_round_up(groups)), dim3(kST * kST),
                       staged_lds_bytes(max_angles), st, src);
    return hipGetLastError();
}

template <int M, class Src>
static hipError_t launch_osl_m(Src src, uint32_t groups, int max_angles, hipStream_t st) {
    static bool once = (allow_large_lds(&kosl_kernel<M, Src>), true);
    (void)once;
    hipLaunchKernelGGL((kosl_kernel<M, Src>), dim3(xcd_round_up(groups)), dim3(kST * kST),
                       staged_lds_bytes(max_angles), st, src);
    return hipGetLastError();
}

hipError_t launch_backproject(int M, const float* y, float* b, float* sens, const ProjArgs& p, hipStream_t st) {
    if (p.A_q > kMaxSubsetAngles) return hipErrorInvalidValue;
    OneJob<BackJob> src{BackJob{p, y, b, sens, 0}};
    const uint32_t g = staged_tile_groups(p.nx, p.ny, p.nz);
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
    return dispatch_osl(M, src, staged_tile_groups(a.g.nx, a.g.ny, a.g.nz), a.g.A_q, st);
}

hipError_t launch_osl_jobs(int M, JobTable<OslJob> jobs, uint32_t groups, int max_angles, hipStream_t st) {
    return dispatch_osl(M, jobs, groups, max_angles, st);
}

}  // namespace kcs
