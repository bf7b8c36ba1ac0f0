// K-back: voxel-driven (gather) back projector and the fused OS-MAP-OSL-KP update.
//
// One thread per voxel.  For each angle of the subset the voxel's footprint on the detector
// covers at most ceil(2 w1 / du) + 1 bins; the exact intersection length of each bin's ray with
// the voxel square (the pixel chord, identical to the Siddon length of that ray in that pixel)
// weights the bin's M-frame record.  The gather needs no atomics and no transposed system
// matrix.  A workgroup covers a 16 x (16 kSV) voxel tile, kSV vertically adjacent voxels per
// thread: for a chunk of the subset's angles it stages in LDS the records of every bin whose ray
// can meet the tile, then each thread gathers for its voxels from LDS, reading a bin its voxels
// share once.  The kernel is latency-bound, so one voxel per thread and a 20 KB staging buffer
// (about 7 workgroups per CU) beat two voxels per thread (fewer LDS reads, but 156 VGPRs).
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

// The same, plus per angle the range of bins whose rays can meet the pixel box (i0, j0, tw, th).
__device__ __forceinline__ void subset_angles_bins_to_lds(AngleRec* sA, int2* sBB, const ProjArgs& p, int i0, int j0,
                                                          int tw, int th) {
    for (int al = threadIdx.x; al < p.A_q; al += blockDim.x) {
        const AngleRec A = make_angle(p.q + al * p.Q, p.n_ang, p.ang0, p.h);
        sA[al] = A;
        int b0, b1;
        box_bins(A, i0, j0, tw, th, p.nx, p.ny, p.h, p.inv_du, p.n_bin, b0, b1);
        sBB[al] = make_int2(b0, b1);
    }
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
__host__ __device__ __forceinline__ void osl_finish(const OslArgs& a, const float* __restrict__ Fm,
                                                    float* __restrict__ x, size_t v, const float (&acc)[M],
                                                    float sens) {
    if (!(sens > 0.0f)) return;  // no ray of this subset sees the voxel: keep x
    const float inv_sens = 1.0f / sens;
    float xv[M];
    load_record<M>(x + v * M, xv);
    if (a.kp) {
        // x b / (n (1 + beta (x - F) / Fe)) = x (acc / sens) Fe / (Fe + beta (x - F)),  Fe = max(F, eps_F);
        // the denominator is at least (1 - beta) Fe > 0, so one hardware reciprocal (1 ulp) serves.
        float F[M];
        load_record<M>(Fm + v * M, F);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float fe = fmaxf(F[m], a.eps_F);
            const float den = fmaf(a.beta_kp, xv[m] - F[m], fe);
            xv[m] = xv[m] * acc[m] * inv_sens * fe * recip(den);
            // eight frames at a time: keeps the scheduler from holding every quotient live at
            // once (all 24 at once need 93 VGPRs and cost two waves per SIMD)
            if (m % 8 == 7) __builtin_amdgcn_sched_barrier(0);
        }
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) xv[m] = xv[m] * acc[m] * inv_sens;
    }
    store_record<M>(x + v * M, xv);
}

template <int M>
__host__ __device__ __forceinline__ void osl_voxel(const AngleRec* sA, const OslArgs& a, const float* __restrict__ ratio,
                                                   const float* __restrict__ Fm, float* __restrict__ x, int i, int j,
                                                   int z) {
    const ProjArgs& p = a.g;
    float acc[M], sens;
    gather<M>(sA, p, ratio, i, j, z, acc, sens);
    osl_finish<M>(a, Fm, x, ((size_t)z * p.ny + j) * p.nx + i, acc, sens);
}

constexpr int kST = 16;                // staged voxel tile: kST columns, one thread per column ...
constexpr int kSV = 1;                 // ... and kSV vertically adjacent voxels per thread
constexpr int kSTY = kST * kSV;        // rows of the staged tile
constexpr int kStageBytes = 20 * 1024;  // LDS for the staged bin records of one angle chunk

// Bins whose rays can meet a w x hgt pixel box: the box's projection is at most
// h sqrt(w^2 + hgt^2) wide, and box_bins widens it by a hundredth of a bin on each side.
__host__ __device__ inline int box_slots(int w, int hgt, float h, float du) {
    return (int)floorf(sqrtf((float)(w * w + hgt * hgt)) * h / du) + 3;
}

// LDS stride of a staged bin record in floats: padded by 4 so that the records of nearby bins,
// which the voxels of a wavefront read at the same time, spread over the banks.
__host__ __device__ constexpr int stage_record(int M) { return M + 4; }

bool staged_fits(int M, float h, float du) {
    return box_slots(kST, kSTY, h, du) * stage_record(M) * (int)sizeof(float) <= kStageBytes;
}

uint32_t staged_tile_groups(int nx, int ny, int nz) {
    return (uint32_t)(((nx + kST - 1) / kST) * ((ny + kSTY - 1) / kSTY)) * nz;
}

// Angles per staging chunk for this geometry.
__host__ __device__ inline int stage_chunk(int M, int slots, int A_q) {
    const int c = kStageBytes / (slots * stage_record(M) * (int)sizeof(float));
    return max(1, min(c, A_q));
}

// For the kSV voxels (i, j + k) of this thread in the staged tile (i0, j0) of plane z:
// acc[k]_m = sum_{d in S_q} p_vd y_dm and sens[k] = sum_{d in S_q} p_vd.  All threads of the
// workgroup must call it (it synchronises).  Per angle the thread walks the union of its voxels'
// detector footprints once, so a bin shared by the voxels is read from LDS once; each voxel takes
// exactly the bins, chords and order of its own footprint.
template <int M>
__device__ __forceinline__ void staged_gather(const AngleRec* sA, const int2* sBB, float4* sR, const ProjArgs& p,
                                              const float* __restrict__ y, int z, int nvalid, int i, int j,
                                              float (&acc)[kSV][M], float (&sens)[kSV]) {
    const int slots = box_slots(kST, kSTY, p.h, p.du);
    const int chunk = stage_chunk(M, slots, p.A_q);
    const float bc = 0.5f * (float)(p.n_bin - 1);
    const float xc = ((float)i - 0.5f * (float)(p.nx - 1)) * p.h;
    float yc[kSV];
#pragma unroll
    for (int k = 0; k < kSV; ++k) {
        yc[k] = ((float)(j + k) - 0.5f * (float)(p.ny - 1)) * p.h;
        sens[k] = 0.0f;
#pragma unroll
        for (int m = 0; m < M; ++m) acc[k][m] = 0.0f;
    }
    const float4* yz = reinterpret_cast<const float4*>(y) + (size_t)z * p.A_q * p.n_bin * (M / 4);
    for (int c0 = 0; c0 < p.A_q; c0 += chunk) {
        const int na = min(chunk, p.A_q - c0);
        __syncthreads();  // previous chunk consumed
        for (int rec = threadIdx.x; rec < na * slots; rec += blockDim.x) {
            const int ar = rec / slots, al = c0 + ar, slot = rec - ar * slots;
            const int2 bb = sBB[al];
            const int b = bb.x + slot;
            if (b > bb.y) continue;
            const float4* src = yz + ((size_t)al * p.n_bin + b) * (M / 4);
            float4* dst = sR + rec * (stage_record(M) / 4);
#pragma unroll
            for (int k = 0; k < M / 4; ++k) dst[k] = src[k];
        }
        __syncthreads();
        if (nvalid == 0) continue;
        for (int ac = 0; ac < na; ++ac) {
            const int al = c0 + ac;
            const AngleRec A = sA[al];
            const int2 bb = sBB[al];
            const int b0 = bb.x, b1 = bb.y;
            const float* ra = reinterpret_cast<const float*>(sR) + (size_t)ac * slots * stage_record(M);
            // each voxel's footprint [lo, hi] as in pixel_footprint, and the union of them
            const float rb = A.w1 * p.inv_du;
            float tc[kSV];
            int lo[kSV], hi[kSV], ulo = p.n_bin, uhi = -1;
#pragma unroll
            for (int k = 0; k < kSV; ++k) {
                tc[k] = fmaf(xc, A.c, yc[k] * A.s);
                const float beta = fmaf(tc[k], p.inv_du, bc);
                lo[k] = max((int)ceilf(beta - rb), 0);
                hi[k] = min((int)floorf(beta + rb), p.n_bin - 1);
                if (k < nvalid) {
                    ulo = min(ulo, lo[k]);
                    uhi = max(uhi, hi[k]);
                }
            }
            for (int b = ulo; b <= uhi; ++b) {
                float len[kSV];
                bool any = false;
#pragma unroll
                for (int k = 0; k < kSV; ++k) {
                    len[k] = (k < nvalid && b >= lo[k] && b <= hi[k]) ? pixel_chord(A, fmaf((float)b - bc, p.du, -tc[k]))
                                                                       : 0.0f;
                    any = any || len[k] > 0.0f;
                }
                if (!any || b < b0 || b > b1) continue;  // b outside [b0, b1] cannot happen: box_bins is a superset
                float v[M];
                load_record<M>(ra + (b - b0) * stage_record(M), v);
#pragma unroll
                for (int k = 0; k < kSV; ++k) {
                    if (len[k] > 0.0f) {
#pragma unroll
                        for (int m = 0; m < M; ++m) acc[k][m] = fmaf(len[k], v[m], acc[k][m]);
                        sens[k] += len[k];
                    }
                }
            }
        }
    }
}

struct StagedTile {
    int i0, j0, z, i, j;
    int nvalid;  // voxels (i, j), (i, j + 1), ... of this thread inside the image
};

__device__ __forceinline__ StagedTile staged_tile(uint32_t w, int nx, int ny, int nz) {
    const int ntx = (nx + kST - 1) / kST, nty = (ny + kSTY - 1) / kSTY;
    StagedTile t;
    t.z = w / (ntx * nty);
    const int r = w % (ntx * nty);
    t.j0 = (r / ntx) * kSTY;
    t.i0 = (r % ntx) * kST;
    t.i = t.i0 + (int)(threadIdx.x % kST);
    t.j = t.j0 + kSV * (int)(threadIdx.x / kST);
    t.nvalid = (t.z < nz && t.i < nx) ? max(0, min(kSV, ny - t.j)) : 0;
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
    int2* sBB = reinterpret_cast<int2*>(lds + (p.A_q * sizeof(AngleRec) + 15) / 16);
    float4* sR = lds + (p.A_q * sizeof(AngleRec) + 15) / 16 + (p.A_q * sizeof(int2) + 15) / 16;
    subset_angles_bins_to_lds(sA, sBB, p, t.i0, t.j0, min(kST, p.nx - t.i0), min(kSTY, p.ny - t.j0));
    float acc[kSV][M], sens[kSV];
    staged_gather<M>(sA, sBB, sR, p, J.y, t.z, t.nvalid, t.i, t.j, acc, sens);
#pragma unroll
    for (int k = 0; k < kSV; ++k) {
        if (k >= t.nvalid) break;
        const size_t v = ((size_t)t.z * p.ny + t.j + k) * p.nx + t.i;
#pragma unroll
        for (int m = 0; m < M; ++m) acc[k][m] *= p.fr.E[m];
        store_record<M>(J.b + v * M, acc[k]);
        if (J.sens) J.sens[v] = sens[k];
    }
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
    int2* sBB = reinterpret_cast<int2*>(lds + (p.A_q * sizeof(AngleRec) + 15) / 16);
    float4* sR = lds + (p.A_q * sizeof(AngleRec) + 15) / 16 + (p.A_q * sizeof(int2) + 15) / 16;
    subset_angles_bins_to_lds(sA, sBB, p, t.i0, t.j0, min(kST, p.nx - t.i0), min(kSTY, p.ny - t.j0));
    float acc[kSV][M], sens[kSV];
    staged_gather<M>(sA, sBB, sR, p, J.ratio, t.z, t.nvalid, t.i, t.j, acc, sens);
#pragma unroll
    for (int k = 0; k < kSV; ++k) {
        if (k >= t.nvalid) break;
        osl_finish<M>(a, J.Fm, J.x, ((size_t)t.z * p.ny + t.j + k) * p.nx + t.i, acc[k], sens[k]);
    }
}

static size_t staged_lds_bytes(int max_angles) {
    return (max_angles * sizeof(AngleRec) + 15) / 16 * 16 + (max_angles * sizeof(int2) + 15) / 16 * 16 + kStageBytes;
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
