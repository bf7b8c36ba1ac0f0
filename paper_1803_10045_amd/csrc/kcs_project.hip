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
    const int b = ray - al * p.n_bin;
    const int a = p.q + al * p.Q;  // global angle index
    const AngleRec A = make_angle(a, p.n_ang, p.ang0, p.h);
    const FrameTab& FT = p.fr;

    float acc[M];
#pragma unroll
    for (int m = 0; m < M; ++m) acc[m] = 0.0f;

    // Ray x c + y s = u in pixel units: X = (x - X0)/h, Y = (y - Y0)/h; point at parameter lam
    // (pixel units of length): X = Xc - lam s, Y = Yc + lam c.
    const float u = ((float)b - 0.5f * (float)(p.n_bin - 1)) * p.du;
    const float Xc = u * A.c * p.inv_h + 0.5f * (float)p.nx;
    const float Yc = u * A.s * p.inv_h + 0.5f * (float)p.ny;
    float lin = -3.0e38f, lout = 3.0e38f;
    bool hit = true;
    if (A.s != 0.0f) {
        const float l0 = Xc * A.inv_s, l1 = (Xc - (float)p.nx) * A.inv_s;
        lin = fmaxf(lin, fminf(l0, l1));
        lout = fminf(lout, fmaxf(l0, l1));
    } else {
        hit = hit && Xc >= 0.0f && Xc < (float)p.nx;
    }
    if (A.c != 0.0f) {
        const float l0 = -Yc * A.inv_c, l1 = ((float)p.ny - Yc) * A.inv_c;
        lin = fmaxf(lin, fminf(l0, l1));
        lout = fminf(lout, fmaxf(l0, l1));
    } else {
        hit = hit && Yc >= 0.0f && Yc < (float)p.ny;
    }
    hit = hit && lout > lin;

    if (hit) {
        // first pixel: the one the ray enters, judged by its direction of travel
        int i, j, si = 0, sj = 0;
        float lx = 3.0e38f, ly = 3.0e38f, dlx = 0.0f, dly = 0.0f;
        if (A.s != 0.0f) {
            const float Xin = Xc - lin * A.s;
            si = A.s < 0.0f ? 1 : -1;
            i = si > 0 ? (int)floorf(Xin) : (int)ceilf(Xin) - 1;
            i = min(max(i, 0), p.nx - 1);
            dlx = fabsf(A.inv_s);
        } else {
            i = (int)floorf(Xc);
        }
        if (A.c != 0.0f) {
            const float Yin = Yc + lin * A.c;
            sj = A.c > 0.0f ? 1 : -1;
            j = sj > 0 ? (int)floorf(Yin) : (int)ceilf(Yin) - 1;
            j = min(max(j, 0), p.ny - 1);
            dly = fabsf(A.inv_c);
        } else {
            j = (int)floorf(Yc);
        }
        // parameters of the next grid-line crossings, re-derived from the line index each step
        const float bx0 = (float)(si > 0 ? i + 1 : i), by0 = (float)(sj > 0 ? j + 1 : j);
        const float lx0 = si ? (Xc - bx0) * A.inv_s : 3.0e38f;
        const float ly0 = sj ? (by0 - Yc) * A.inv_c : 3.0e38f;
        int kx = 0, ky = 0;
        lx = lx0;
        ly = ly0;
        float lcur = lin;
        const float* plane = x + (size_t)z * p.nx * p.ny * M;
        const int max_steps = p.nx + p.ny + 2;
        for (int step = 0; step < max_steps; ++step) {
            const float lnext = fminf(fminf(lx, ly), lout);
            const float len = (lnext - lcur) * p.h;
            float v[M];
            load_record<M>(plane + ((size_t)j * p.nx + i) * M, v);
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] = fmaf(len, v[m], acc[m]);
            if (lnext >= lout) break;
            if (lx <= ly) {
                i += si;
                ++kx;
                lx = fmaf((float)kx, dlx, lx0);
            } else {
                j += sj;
                ++ky;
                ly = fmaf((float)ky, dly, ly0);
            }
            if (i < 0 || i >= p.nx || j < 0 || j >= p.ny) break;
            lcur = lnext;
        }
    }

    const size_t o = (((size_t)z * p.A_q + al) * p.n_bin + b) * M;
    float y[M];
    if (RATIO) {
        float s[M];
        load_record<M>(sino + (((size_t)z * p.n_ang + a) * p.n_bin + b) * M, s);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float yb = fmaf(FT.E[m], acc[m], FT.r[m]);
            y[m] = yb > 0.0f ? s[m] / yb : 0.0f;
        }
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) y[m] = fmaf(FT.E[m], acc[m], FT.r[m]);
    }
    store_record<M>(out + o, y);
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
