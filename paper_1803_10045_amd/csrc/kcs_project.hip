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
// tile (a group of frames) in LDS per workgroup and traverses, inside the tile, every subset ray
// that can meet it, writing one partial line integral per (tile, ray, frame group).
// kproj_reduce_kernel adds the partials of each ray over the tiles in a fixed order
// (deterministic, no atomics) and applies the same epilogue.  The image then crosses HBM once per
// subset; the partials cost about 2 x image x 16 / T bytes, so larger tiles (with fewer frames
// staged per workgroup) move less.
//
// All kernels take a job source: one study by value, or a device table of studies.
#include "kcs_device.h"
#include "kcs_launch.h"

namespace kcs {

// A point of ray (FP64 cos c, sin s of its angle; bin b0) near the centre (cx, cy) of a pixel box whose corner is pixel
// (i0, j0), in pixel units relative to that corner, computed in FP64 and rounded to FP32.  The
// ray's position is known to the FP64 rounding of the geometry, and near the box the FP32 point
// carries an error of the order of ulp(box size) instead of ulp(distance to the image centre):
// the corner chords of pixels far from the centre then keep their FP64 lengths to ~1e-6 pixel.
__host__ __device__ inline float2 ray_point_near(double c, double s, int b0, const ProjArgs& p, int i0, int j0,
                                                 double cx, double cy) {
    const double u = ((double)b0 - 0.5 * (double)(p.n_bin - 1)) * p.dud / p.hd;  // pixel units
    const double X = u * c + 0.5 * (double)p.nx - (double)i0;  // foot point of the ray's normal
    const double Y = u * s + 0.5 * (double)p.ny - (double)j0;
    const double lam = (cx - X) * -s + (cy - Y) * c;  // along the ray direction (-s, c)
    return make_float2((float)(X - lam * s), (float)(Y + lam * c));
}

// Expected counts or measured/expected ratio of ray (z, al, b) from its line integrals acc:
// ybar_m = E_m mu acc_m + r_m, mu the ray's multiplicative correction (1 without one).
template <int M, bool RATIO>
__host__ __device__ __forceinline__ void ray_epilogue(const ProjArgs& p, const float* __restrict__ sino,
                                                      float* __restrict__ out, int z, int al, int b,
                                                      const float (&acc)[M]) {
    const int a = p.q + al * p.Q;
    const size_t o = (((size_t)z * p.A_q + al) * p.n_bin + b) * M;
    const size_t ray = ((size_t)z * p.n_ang + a) * p.n_bin + b;
    const float mu = p.mult ? p.mult[ray] : 1.0f;
    float y[M];
    if (RATIO) {
        float s[M];
        load_record<M>(sino + ray * M, s);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float yb = fmaf(p.fr.E[m] * mu, acc[m], p.fr.r[m]);
            y[m] = yb > 0.0f ? s[m] / yb : 0.0f;
        }
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) y[m] = fmaf(p.fr.E[m] * mu, acc[m], p.fr.r[m]);
    }
    store_record<M>(out + o, y);
}

// Ray (z, al, b) of subset p.q through the whole plane.
template <int M, bool RATIO>
__host__ __device__ __forceinline__ void project_ray(const ProjArgs& p, const float* __restrict__ x,
                                                     const float* __restrict__ sino, float* __restrict__ out, int z,
                                                     int al, int b) {
    double c, s;
    angle_cos_sin(p.q + al * p.Q, p.n_ang, p.ang0, c, s);
    const AngleRec A = make_angle_cs(c, s, p.h);
    float acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0f;
    // the ray's point nearest the image centre, in pixel units from the image corner
    const float2 pt = ray_point_near(c, s, b, p, 0, 0, 0.5 * p.nx, 0.5 * p.ny);
    const float* plane = x + (size_t)z * p.nx * p.ny * M;
    siddon_traverse_box(A, pt.x, pt.y, p.nx, p.ny, p.h, p.nx * M, M, [&](int idx, float len) {
        float v[M];
        load_record<M>(plane + idx, v);
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] = fmaf(len, v[m], acc[m]);
    });
    ray_epilogue<M, RATIO>(p, sino, out, z, al, b, acc);
}

uint32_t proj_direct_groups(const ProjArgs& p) { return (uint32_t)((p.rays_per_plane + 255) / 256) * p.nz; }

// Lanes per ray of the reduce step of a tiled projection (a power of 2 dividing 64): a ray's
// partial sums lie in about one tile per tile row, so the lanes split the rows and more loads are
// in flight than with one lane walking all of them.
constexpr int kReduceLanes = 4;

uint32_t proj_reduce_groups(const ProjArgs& p) {
    return (uint32_t)(((int64_t)p.rays_per_plane * kReduceLanes + 255) / 256) * p.nz;
}

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

// Tile variants: a T x T pixel tile with FG = M / NG of its frames staged in LDS per workgroup
// (NG frame groups; the groups of one tile are adjacent work items, so they share the tile's
// cache lines in L2).  Larger tiles cut the partial sums (a ray leaves one partial per tile it
// crosses); fewer groups walk each ray segment fewer times.  Each staged tile stays within
// 80 KB, so that two workgroups share a CU and one stages while the other walks (measured: a
// whole-record 32-pixel tile, one workgroup per CU, walks each segment once but runs slower).
// LDS row stride of a staged tile in floats: padded by 4 so that vertically adjacent pixels,
// which parallel rays of a near-horizontal angle read at the same step, fall in other banks.
__host__ __device__ constexpr int tile_row(int T, int FG) { return T * FG + 4; }
__host__ __device__ constexpr size_t tile_lds_bytes(int T, int FG) { return (size_t)T * tile_row(T, FG) * sizeof(float); }
__host__ __device__ constexpr int tile_threads(int T) { return T == 16 ? 256 : 512; }
constexpr size_t kLdsBytes = 160 * 1024;  // LDS of a CU

// Frame groups of the tiled projector for M frames and tile T: the fewest whose staged tile
// leaves room for two workgroups per CU (one stages its tile while the other walks).
__host__ __device__ constexpr int tile_groups_for(int M, int T) {
    return tile_lds_bytes(T, M) <= 80 * 1024 ? 1 : (M % 8 == 0 && tile_lds_bytes(T, M / 2) <= 80 * 1024 ? 2 : M / 4);
}

uint32_t proj_tile_groups(const ProjArgs& p, int T) {
    return (uint32_t)(((p.nx + T - 1) / T) * ((p.ny + T - 1) / T)) * p.nz * tile_groups_for(p.fr.M, T);
}

size_t tile_partial_bytes(int T, const ProjArgs& p, int M) {
    const size_t ntx = (p.nx + T - 1) / T, nty = (p.ny + T - 1) / T;
    return (size_t)p.nz * ntx * nty * p.A_q * tile_slots(T, p.h, p.du) * M * sizeof(float);
}

// FG consecutive floats (FG even; 8-byte aligned, 16-byte aligned when FG % 4 == 0).
template <int FG>
__host__ __device__ __forceinline__ void load_frames(const float* __restrict__ p, float (&v)[FG]) {
    if constexpr (FG % 4 == 0) {
#pragma unroll
        for (int k = 0; k < FG / 4; ++k) {
            const float4 q = reinterpret_cast<const float4*>(p)[k];
            v[4 * k] = q.x;
            v[4 * k + 1] = q.y;
            v[4 * k + 2] = q.z;
            v[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < FG / 2; ++k) {
            const float2 q = reinterpret_cast<const float2*>(p)[k];
            v[2 * k] = q.x;
            v[2 * k + 1] = q.y;
        }
    }
}

template <int FG>
__host__ __device__ __forceinline__ void store_frames(float* __restrict__ p, const float (&v)[FG]) {
    if constexpr (FG % 4 == 0) {
#pragma unroll
        for (int k = 0; k < FG / 4; ++k)
            reinterpret_cast<float4*>(p)[k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < FG / 2; ++k) reinterpret_cast<float2*>(p)[k] = make_float2(v[2 * k], v[2 * k + 1]);
    }
}

// Partial sums: psum[g][tile][angle][slot][FG] for frame group g, tile (z, ty, tx) in plane-major
// order; each workgroup writes a dense block.
__host__ __device__ __forceinline__ size_t partial_offset(int g, size_t n_tiles, size_t tile, int A_q, int al,
                                                          int slots, int slot, int FG) {
    return ((((size_t)g * n_tiles + tile) * A_q + al) * slots + slot) * FG;
}

// Per-angle LDS table of the tile kernel: the angle's constants, the bins [b0, b1] whose rays
// can meet the tile, and a point of ray b0 near the tile centre (see ray_point_near).
struct TileAngle {
    AngleRec A;
    int32_t b0, b1;
    float px, py;
};

// The angle al of work item it: start[al] <= it < start[al + 1] (binary search over the LDS table).
__device__ __forceinline__ int item_angle(const int* start, int A_q, int it) {
    int lo = 0, hi = A_q - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int M, int T, int NG, class Src>
__global__ __launch_bounds__(tile_threads(T)) void kproj_tile_kernel(Src src) {
    constexpr int FG = M / NG, NT = tile_threads(T), TS = tile_row(T, FG);
    static_assert(M % FG == 0 && FG % 4 == 0, "frame groups");
    extern __shared__ float4 lds4[];
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const ProjJob& J = src.find(w);
    const ProjArgs& p = J.p;
    const int slots = J.slots;
    float* tile = reinterpret_cast<float*>(lds4);
    TileAngle* sT = reinterpret_cast<TileAngle*>(lds4 + T * TS / 4);
    const int ntx = (p.nx + T - 1) / T, nty = (p.ny + T - 1) / T;
    const uint32_t lw = w - J.w0;
    const int g = (int)(lw % NG);
    const uint32_t tl = lw / NG;
    const int z = tl / (ntx * nty);
    if (z >= p.nz) return;  // whole workgroup
    const int tr = tl % (ntx * nty), ty = tr / ntx, tx = tr % ntx;
    const int i0 = tx * T, j0 = ty * T, tw = min(T, p.nx - i0), th = min(T, p.ny - j0);
    // stage frame group g of the tile: pixel (r, c) -> tile[r * TS + c * FG]
    const float* src_px = J.x + (((size_t)z * p.ny + j0) * p.nx + i0) * M + g * FG;
    for (int e = threadIdx.x; e < th * tw; e += NT) {
        const int r = e / tw, c = e - r * tw;
        float v[FG];
        load_frames<FG>(src_px + ((size_t)r * p.nx + c) * M, v);
        store_frames<FG>(tile + r * TS + c * FG, v);
    }
    // start[al] = first work item of angle al (items are the bins of each angle that can meet the
    // tile, angle after angle); start[A_q] = number of items
    int* start = reinterpret_cast<int*>(sT + p.A_q);
    for (int al = threadIdx.x; al < p.A_q; al += NT) {
        TileAngle t;
        double c, s;
        angle_cos_sin(p.q + al * p.Q, p.n_ang, p.ang0, c, s);
        t.A = make_angle_cs(c, s, p.h);
        box_bins(t.A, i0, j0, tw, th, p.nx, p.ny, p.h, p.inv_du, p.n_bin, t.b0, t.b1);
        const float2 pt = ray_point_near(c, s, t.b0, p, i0, j0, 0.5 * tw, 0.5 * th);
        t.px = pt.x;
        t.py = pt.y;
        sT[al] = t;
        start[al + 1] = min(max(t.b1 - t.b0 + 1, 0), slots);
    }
    __syncthreads();
    if (threadIdx.x < 64) {  // inclusive scan of the counts by the first wave, 64 angles at a time
        int carry = 0;
        for (int base = 0; base < p.A_q; base += 64) {
            const int al = base + (int)threadIdx.x;
            int v = al < p.A_q ? start[al + 1] : 0;
#pragma unroll
            for (int d = 1; d < 64; d *= 2) {
                const int u = __shfl_up(v, d, 64);
                if ((int)threadIdx.x >= d) v += u;
            }
            if (al < p.A_q) start[al + 1] = v + carry;
            carry += __shfl(v, 63, 64);
        }
        if (threadIdx.x == 0) start[0] = 0;
    }
    __syncthreads();
    const int n_items = start[p.A_q];
    const size_t n_tiles = (size_t)p.nz * nty * ntx;
    float* out = J.psum + partial_offset(g, n_tiles, (size_t)z * nty * ntx + tr, p.A_q, 0, slots, 0, FG);
    const float bin_step = p.du * p.inv_h;  // bin width in pixel units
    // Work items: one ray segment each, angle after angle (a wave's lanes walk parallel rays of
    // one or two angles through the tile, so their LDS reads stay close); only bins that can meet
    // the tile are items.
    for (int it = threadIdx.x; it < n_items; it += NT) {
        const int al = item_angle(start, p.A_q, it), slot = it - start[al];
        const TileAngle ta = sT[al];
        float acc[FG];
#pragma unroll
        for (int m = 0; m < FG; ++m) acc[m] = 0.0f;
        // a point of ray b0 + slot: ray b0's point moved `slot` bins along the detector normal
        const float off = (float)slot * bin_step;
        const float Xc = fmaf(off, ta.A.c, ta.px), Yc = fmaf(off, ta.A.s, ta.py);
        // pixel offsets in bytes, so that the LDS address needs no scaling per crossing
        siddon_traverse_box(ta.A, Xc, Yc, tw, th, p.h, TS * 4, FG * 4, [&](int o, float len) {
            float v[FG];
            load_frames<FG>(reinterpret_cast<const float*>(reinterpret_cast<const char*>(tile) + o), v);
#pragma unroll
            for (int m = 0; m < FG; ++m) acc[m] = fmaf(len, v[m], acc[m]);
        });
        store_frames<FG>(out + ((size_t)al * slots + slot) * FG, acc);
    }
}

template <int M, int T, int NG, bool RATIO, class Src>
__global__ __launch_bounds__(256) void kproj_reduce_kernel(Src src) {
    constexpr int FG = M / NG;
    const uint32_t w = xcd_work_index(blockIdx.x, gridDim.x);
    const ProjJob& J = src.find(w);
    const ProjArgs& p = J.p;
    const int slots = J.slots;
    const uint32_t lw = w - J.w0;
    const uint32_t blocks_per_plane = (p.rays_per_plane * kReduceLanes + 255u) / 256u;
    const uint32_t z = lw / blocks_per_plane;
    if (z >= (uint32_t)p.nz) return;
    // kReduceLanes adjacent lanes share a ray (all of them in range or none), each summing the
    // tile rows ty = part, part + kReduceLanes, ...; their sums are added by a butterfly below
    const uint32_t lane_id = (lw % blocks_per_plane) * 256u + threadIdx.x;
    const uint32_t ray = lane_id / kReduceLanes;
    const int part = (int)(lane_id % kReduceLanes);
    if (ray >= (uint32_t)p.rays_per_plane) return;
    const int al = ray / p.n_bin;
    const int b = ray - al * p.n_bin;
    const AngleRec A = make_angle(p.q + al * p.Q, p.n_ang, p.ang0, p.h);
    const int ntx = (p.nx + T - 1) / T, nty = (p.ny + T - 1) / T;
    const size_t n_tiles = (size_t)p.nz * nty * ntx;
    float acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0f;
    // Along a row of tiles the projection of a full-width tile moves by `slope` bins per column,
    // so the columns whose bin range can hold b form an interval; it is found from the row's
    // first tile and widened by one column on each side, and box_bins, the producer's own test,
    // then decides for each column in it (a last, narrower tile projects inside the full-width
    // one, so the interval still covers it).
    const float slope = (float)T * p.h * A.c * p.inv_du;
    const float bc = 0.5f * (float)(p.n_bin - 1);
    for (int ty = part; ty < nty; ty += kReduceLanes) {
        int lo = 0, hi = ntx - 1;
        if (fabsf(slope) > 1e-3f) {
            const float xl = -0.5f * (float)p.nx * p.h, xr = xl + (float)T * p.h;
            const float yl = ((float)(ty * T) - 0.5f * (float)p.ny) * p.h, yr = yl + (float)min(T, p.ny - ty * T) * p.h;
            const float umin = fminf(xl * A.c, xr * A.c) + fminf(yl * A.s, yr * A.s);
            const float umax = fmaxf(xl * A.c, xr * A.c) + fmaxf(yl * A.s, yr * A.s);
            const float ta = ((float)b - fmaf(umax, p.inv_du, bc) - 0.01f) / slope;
            const float tb = ((float)b - fmaf(umin, p.inv_du, bc) + 0.01f) / slope;
            const float lim = (float)ntx + 2.0f;
            lo = max(lo, (int)floorf(fminf(fmaxf(fminf(ta, tb), -lim), lim)) - 1);
            hi = min(hi, (int)ceilf(fminf(fmaxf(fmaxf(ta, tb), -lim), lim)) + 1);
        }
        for (int tx = lo; tx <= hi; ++tx) {
            const int i0 = tx * T, j0 = ty * T;
            int b0, b1;
            box_bins(A, i0, j0, min(T, p.nx - i0), min(T, p.ny - j0), p.nx, p.ny, p.h, p.inv_du, p.n_bin, b0, b1);
            if (b < b0 || b > b1 || b - b0 >= slots) continue;
            const size_t t = ((size_t)z * nty + ty) * ntx + tx;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                float v[FG];
                load_frames<FG>(J.psum + partial_offset(g, n_tiles, t, p.A_q, al, slots, b - b0, FG), v);
#pragma unroll
                for (int m = 0; m < FG; ++m) acc[g * FG + m] += v[m];
            }
        }
    }
    // every lane of the ray ends with the same total (a + b == b + a exactly)
#pragma unroll
    for (int d = 1; d < kReduceLanes; d *= 2)
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] += __shfl_xor(acc[m], d, 64);
    if (part == 0) ray_epilogue<M, RATIO>(p, J.sino, J.out, z, al, b, acc);
}

// ---------------------------------------------------------------------------------------------
// Launch helpers

template <int M, int T, int NG, class Src>
static hipError_t launch_tile(Src src, uint32_t groups, int max_angles, hipStream_t st) {
    constexpr int FG = M / NG;
    static bool attr_set = false;  // the tile may exceed the default 64 KB of dynamic LDS
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&kproj_tile_kernel<M, T, NG, Src>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
        attr_set = true;
    }
    const size_t lds = tile_lds_bytes(T, FG) + (size_t)max_angles * sizeof(TileAngle) + (size_t)(max_angles + 1) * sizeof(int);
    if (lds > kLdsBytes) return hipErrorInvalidValue;
    hipLaunchKernelGGL((kproj_tile_kernel<M, T, NG, Src>), dim3(xcd_round_up(groups)), dim3(tile_threads(T)), lds,
                       st, src);
    return hipGetLastError();
}

template <int M, int T, int NG, class Src>
static hipError_t launch_reduce(Src src, uint32_t groups, bool ratio, hipStream_t st) {
    if (ratio)
        hipLaunchKernelGGL((kproj_reduce_kernel<M, T, NG, true, Src>), dim3(xcd_round_up(groups)), dim3(256), 0, st, src);
    else
        hipLaunchKernelGGL((kproj_reduce_kernel<M, T, NG, false, Src>), dim3(xcd_round_up(groups)), dim3(256), 0, st,
                           src);
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

// Whether the T x T tile with M / NG frames per group is built: whole 4-float groups, two
// workgroups per CU.
template <int M, int T, int NG>
constexpr bool tile_built() {
    return M % NG == 0 && (M / NG) % 4 == 0 && tile_lds_bytes(T, M / NG) <= 80 * 1024;
}

template <int M, int T, int NG, class Src>
static hipError_t tile_or_reduce(Src src, uint32_t groups, int max_angles, bool ratio, bool reduce_step, hipStream_t st) {
    if constexpr (tile_built<M, T, NG>())
        return reduce_step ? launch_reduce<M, T, NG>(src, groups, ratio, st) : launch_tile<M, T, NG>(src, groups, max_angles, st);
    else
        return hipErrorInvalidValue;
}

// One step of the projector for frame count M and tile T (T = 0: ray-driven): the tile step
// (reduce_step = false) or the reduce step of a tiled projection, or the ray-driven kernel.
template <int M, class Src>
static hipError_t project_step(int T, Src src, uint32_t groups, int max_angles, bool ratio, bool reduce_step,
                               hipStream_t st) {
    switch (T) {
        case 0: return reduce_step ? hipSuccess : launch_direct<M>(src, groups, ratio, st);
        case 16: return tile_or_reduce<M, 16, tile_groups_for(M, 16)>(src, groups, max_angles, ratio, reduce_step, st);
        case 32: return tile_or_reduce<M, 32, tile_groups_for(M, 32)>(src, groups, max_angles, ratio, reduce_step, st);
        case 64: return tile_or_reduce<M, 64, tile_groups_for(M, 64)>(src, groups, max_angles, ratio, reduce_step, st);
        default: return hipErrorInvalidValue;
    }
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
    if (T != 16 && T != 32 && T != 64) return hipErrorInvalidValue;
    OneJob<ProjJob> src{ProjJob{p, x, sino, out, psum, tile_slots(T, p.h, p.du), 0}};
    hipError_t e = dispatch_project(M, T, src, proj_tile_groups(p, T), p.A_q, ratio, false, st);
    if (e != hipSuccess) return e;
    return dispatch_project(M, T, src, proj_reduce_groups(p), p.A_q, ratio, true, st);
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
