/*
 * kcs.h -- kinetic compressive sensing (direct parametric PET reconstruction) on MI355X.
 *
 * C ABI of libkcs.so.  One ICM sweep (Sec. II-D) alternates
 *   (a) an ordered-subsets MAP one-step-late activity update with the kinetics-derived prior
 *       (Eq. 2 with the potential of Eq. 3), and
 *   (b) a per-voxel MAP Levenberg-Marquardt fit of the irreversible two-tissue model with the
 *       Huber prior on neighbour differences of the kinetic maps (Eq. 4-7).
 *
 * Conventions shared by every entry point
 *   - Device arrays are FP32, C order, owned and allocated by the caller; the library never
 *     frees them.  The time-frame index is innermost:
 *       image x        [nz][ny][nx][M]      (frame-mean activity, units of the input function)
 *       sinogram s     [nz][n_ang][n_bin][M] (counts)
 *       subset sinogram[nz][A_q][n_bin][M]   (A_q = angles of subset q, see below)
 *       kinetic maps   [3][nz][ny][nx]      (K1, k2, k3 planes, "structure of arrays")
 *       damping lambda [nz][ny][nx]
 *   - Host arrays (frame schedule, scales) are FP64 and only read during the call.
 *   - Every call is asynchronous on `stream` (0 = the null stream) and never synchronises the
 *     device.  Arguments are validated on the host before anything is launched, so a call
 *     that returns an error has no side effect.  Return value: KCS_OK or a negative code;
 *     kcs_last_error() gives a message for the calling thread.
 *   - Calls that need the kinetic-model constants (everything but kcs_project / kcs_backproject)
 *     build them with a small FP64 kernel in the caller's workspace, so no host-to-device copy is
 *     made and every call only enqueues kernels (and device-to-device copies) on `stream`.
 *   - Calls sharing a workspace must be ordered (same stream, or synchronised); the workspace
 *     must be 256-byte aligned.
 *   - M (frames) must be one of 8, 16, 24, 32.
 *
 * Geometry: 2D parallel-beam projections of direct planes.  Pixels are squares of side
 * pixel_mm centred at ((i - (nx-1)/2) h, (j - (ny-1)/2) h).  Ray (a, b) is the line
 * x cos(t_a) + y sin(t_a) = u_b with t_a = ang0_rad + a pi / n_ang and
 * u_b = (b - (n_bin-1)/2) bin_mm.  The system matrix element p_vd (Eq. 2) is the exact length
 * (mm) of ray d inside pixel v (Siddon's radiological path).  Ordered subset q of Q holds the
 * angles a with a mod Q = q, in increasing order (A_q = ceil((n_ang - q) / Q) of them).
 */
#ifndef KCS_H
#define KCS_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    KCS_OK = 0,
    KCS_EINVAL = -1,     /* null pointer, non-positive size, unsorted frames, bad value */
    KCS_ESHAPE = -2,     /* shape the library does not support (M not in {8,16,24,32}, more than 1024
                            angles in a subset, bins more than 6 times narrower than pixels, a plane of
                            nx*ny*M >= 2^31 values) */
    KCS_EWORKSPACE = -3, /* workspace smaller than kcs_workspace_bytes() */
    KCS_EHIP = -4        /* HIP runtime error (message has hipGetErrorString) */
};

typedef struct kcs_geometry {
    int32_t nx, ny, nz; /* image grid, >= 1 each, nx*ny*nz < 2^31 and nx*ny*M < 2^31 (M frames) */
    double pixel_mm;    /* in-plane square pixel side h > 0 */
    int32_t n_ang;      /* projection angles over 180 degrees, >= 1 */
    int32_t n_bin;      /* radial bins per angle, >= 1 */
    double bin_mm;      /* radial bin width > 0 */
    double ang0_rad;    /* angle of projection 0 */
    /* Multiplicative correction sinogram [nz][n_ang][n_bin] (device, read only, caller-owned):
     * the product of the attenuation factor and the detector-pair efficiency of each ray, finite
     * and >= 0 (the acquisition model of Sec. II-A includes attenuation).  The system matrix becomes diag(d_mult) P: every projection, back projection and
     * sensitivity below is weighted by it.  NULL means all ones (no attenuation, uniform
     * efficiencies).  The library reads only the rays it projects. */
    const float* d_mult;
} kcs_geometry;

typedef struct kcs_frames {
    int32_t n_frames;     /* M */
    const double* t0_min; /* host [M] frame start, minutes, >= 0; a start within 1e-12 (relative) of the
                             previous frame's end is taken as that end (frames then share a boundary) */
    const double* t1_min; /* host [M] frame end, > start, frames sorted and non-overlapping */
    const double* scale;  /* host [M] E_m = c * (t1_m - t0_m): expected counts per activity unit per mm of path */
    const double* bg;     /* host [M] r_m >= 0: flat additive background, counts per bin (randoms + scatter) */
} kcs_frames;

/* Plasma input Cp(t) = (A1 t - A2 - A3) e^{l1 t} + A2 e^{l2 t} + A3 e^{l3 t} (t >= 0, minutes;
 * Cp = 0 before 0) and the measured TAC model C_PET = (1 - vb) C_T + vb Cp with the irreversible
 * two-tissue tissue curve C_T(K1, k2, k3) (k4 = 0).  l1 < l2 < l3 < 0 distinct.
 * fit_vb = 0: vb is the study's blood fraction, 0 <= vb < 1, and the kinetic maps are the three
 * maps [3][nz][ny][nx] (K1, k2, k3).  fit_vb = 1: the blood fraction is a fourth map per voxel
 * (the f_v map of Sec. IV and Table I), the maps are [4][nz][ny][nx] (K1, k2, k3, vb) everywhere
 * below (model TAC, OSL prior, MAP-LM fit, initial state), and the field vb is not used.  Plans do
 * not take fit_vb = 1 (KCS_EINVAL). */
typedef struct kcs_kinetics {
    double A1, A2, A3, l1, l2, l3, vb;
    int32_t fit_vb;
} kcs_kinetics;

/* Priors.  OSL denominator (Eq. 2-3): D = n (1 + beta_kp (x - F) / max(F, eps_F)) with
 * 0 <= beta_kp < 1 and eps_F > 0; kp_on = 0 turns the kinetics-derived prior off (plain OS-EM).
 * MAP-LM (Eq. 4-7): weight beta_h >= 0 and Huber threshold delta[p] > 0 per kinetic map (delta[3],
 * of the blood-fraction map, only read with kcs_kinetics.fit_vb).
 * Neighbourhood of the Huber term: plane_ratio = 0 takes the 8 in-plane neighbours (the paper's
 * prior, weights 1 and 1/sqrt(2)); plane_ratio > 0 takes the 26 neighbours of the 3x3x3 cube,
 * the planes being plane_ratio pixel sides apart, each weighted by 1 / its distance in pixel
 * sides.  plane_ratio must be finite and >= 0. */
typedef struct kcs_prior {
    double beta_kp, eps_F, beta_h, delta[4];
    int32_t kp_on;
    double plane_ratio;
} kcs_prior;

/* Levenberg-Marquardt schedule: n_iter synchronous iterations; lambda <= 0 on entry is set to
 * tau * max diag(J^T J); parameters clipped to [lo, hi] (lo[1] + lo[2] > 0; the blood fraction's
 * bounds lo[3], hi[3] are read only with fit_vb and must satisfy 0 <= lo[3] <= hi[3] <= 1); a step is accepted
 * iff the voxel objective decreases by more than eta times its value,
 * Phi(xi') - Phi(xi) < -eta Phi(xi) (0 <= eta < 1; eta = 0 is the plain strict decrease), then
 * lambda = max(lambda/10, lam_min), otherwise lambda = min(10 lambda, lam_max).
 * restart (ICM sweeps and plans only): non-zero starts every sweep's fit from
 * tau * max diag(J^T J) whatever d_lambda holds (each sweep fits a new image); zero continues
 * from d_lambda, the damping the previous sweep's fit left (lambda <= 0 still initialises).
 * kcs_lm_fit always starts from d_lambda. */
typedef struct kcs_lm_opts {
    int32_t n_iter;
    double tau, lam_min, lam_max, lo[4], hi[4], eta;
    int32_t restart;
} kcs_lm_opts;

/* Bytes of device workspace the calls below need for this geometry, frame count and subset count. */
size_t kcs_workspace_bytes(const kcs_geometry* g, int32_t n_frames, int32_t Q);

/* Device bytes one study occupies: sinogram, image, three maps, lambda, workspace and, when
 * g->d_mult is given, the correction sinogram (nz * n_ang * n_bin floats). */
size_t kcs_study_footprint_bytes(const kcs_geometry* g, int32_t n_frames, int32_t Q);

/* Expected counts of subset q (denominator of Eq. 2 plus background):
 *   ybar_dm = E_m sum_v p_vd x_vm + r_m   for the rays d of subset q.
 * d_x: image [nz][ny][nx][M]; d_ybar: [nz][A_q][n_bin][M] (written).  0 <= q < Q <= n_ang. */
int kcs_project(const kcs_geometry* g, const kcs_frames* f, const float* d_x, int32_t q, int32_t Q,
                float* d_ybar, hipStream_t stream);

/* Adjoint of the linear part of kcs_project (outer sum of Eq. 2):
 *   b_vm = E_m sum_{d in S_q} p_vd y_dm,   sens_v = sum_{d in S_q} p_vd.
 * d_y: [nz][A_q][n_bin][M]; d_b: [nz][ny][nx][M] (written); d_sens: [nz][ny][nx] or NULL. */
int kcs_backproject(const kcs_geometry* g, const kcs_frames* f, const float* d_y, int32_t q, int32_t Q,
                    float* d_b, float* d_sens, hipStream_t stream);

/* Net uptake rate map (the macro-parameter of Sec. IV, human data): for each of n voxels
 *   K_i = K1 k3 / (k2 + k3),   and K_i = K1 where k2 + k3 = 0 (nothing leaves the first
 *   compartment, so everything that enters is taken up).
 * d_params: [3][n] device maps (K1, k2, k3), read; d_ki: [n] device, written.  Caller-owned.
 * Errors: KCS_EINVAL for n < 0, n > (2^31 - 1) * 256 or a NULL pointer with n > 0 (nothing is
 * launched); n = 0 is a no-op.  Asynchronous on `stream`; needs no workspace. */
int kcs_ki_map(const float* d_params, int64_t n, float* d_ki, hipStream_t stream);

/* Single-slice rebinning of a 3D acquisition (Sec. IV: the human study's 3D listmode data are
 * rebinned into the sinograms this reconstruction takes).  A scanner of R rings records a
 * sinogram for every ring pair (r1, r2) with |r2 - r1| <= D; the axial midpoint of its lines of
 * response lies on plane z = r1 + r2 of the 2R - 1 planes spaced half a ring apart (direct planes
 * at even z, cross planes at odd z), and the rebinning adds it there:
 *   y2d[z][a][b][m] = sum over delta = -D..D, in increasing order, with z - delta even,
 *                     r1 = (z - delta) / 2 and r2 = r1 + delta both in [0, R):
 *                     y3d[delta + D][r1][a][b][m];
 *   count[z] = the number of those ring pairs (the plane's sensitivity in units of one
 *              sinogram: a factor of the plane's multiplicative correction, kcs_geometry.d_mult).
 * d_y3d: [2D + 1][R][n_ang][n_bin][n_frames] device, span 1, indexed by ring difference and first
 * ring (entries of ring pairs outside the scanner are not read); d_y2d: [2R - 1][n_ang][n_bin]
 * [n_frames] device, written; d_count: [2R - 1] device floats, written, or NULL.  Sums in FP32
 * (exact for integer counts below 2^24).  Caller-owned buffers; asynchronous on `stream`.
 * Errors (nothing launched): KCS_EINVAL for R outside [1, 4096], D outside [0, R - 1], n_ang,
 * n_bin or n_frames < 1, or a NULL d_y3d / d_y2d; KCS_ESHAPE for an output of 2^40 or more
 * values. */
int kcs_rebin_ssrb(int32_t n_rings, int32_t max_ring_diff, int32_t n_ang, int32_t n_bin, int32_t n_frames,
                   const float* d_y3d, float* d_y2d, float* d_count, hipStream_t stream);

/* Frame-averaged model TAC (Eq. 3's F(xi)_m, closed-form time integrals) for n voxels:
 *   F_m = (1/dt_m) int_{t0_m}^{t1_m} [(1 - vb) C_T(t; K1, k2, k3) + vb Cp(t)] dt
 * d_params: [P][n] (K1, k2, k3 with k2 + k3 > 0, and vb with k->fit_vb; P = 3 or 4); d_F: [n][M];
 * d_J: [n][M][P] dF/d(K1, k2, k3[, vb]) or NULL.
 * d_work: at least kcs_workspace_bytes(NULL, M, 0) bytes. */
int kcs_model_tac(const kcs_frames* f, const kcs_kinetics* k, const float* d_params, int64_t n, float* d_F,
                  float* d_J, void* d_work, size_t work_bytes, hipStream_t stream);

/* One OS-MAP-OSL-KP update with subset q (Eq. 2 with the potential of Eq. 3):
 *   x_vm <- x_vm * b_vm / D_vm,  b_vm = E_m sum_{d in S_q} p_vd s_dm / ybar_dm,
 *   D_vm = n_vm [1 + beta_kp (x_vm - F_vm) / max(F_vm, eps_F)] (prior on) or n_vm (off),
 *   n_vm = E_m sum_{d in S_q} p_vd;  x unchanged where n_vm = 0;  F from d_params.
 * d_sino: measured [nz][n_ang][n_bin][M]; d_params: [3][nz][ny][nx]; d_x updated in place. */
int kcs_osl_update(const kcs_geometry* g, const kcs_frames* f, const kcs_kinetics* k, const kcs_prior* p,
                   const float* d_sino, const float* d_params, int32_t q, int32_t Q, float* d_x, void* d_work,
                   size_t work_bytes, hipStream_t stream);

/* lm->n_iter synchronous MAP-LM iterations (Eq. 4-7) on every voxel of the image d_x:
 *   g = J^T (x - F) - beta_h sum_k w_k psi(xi_v - xi_k),  step = (J^T J + lambda I)^{-1} g,
 * trial clipped to [lo, hi] and kept iff the voxel's objective decreases by more than eta times
 * its value (kcs_lm_opts); neighbours k are the in-plane 8-neighbourhood (w = 1 edge, 1/sqrt 2
 * diagonal) or, with p->plane_ratio > 0, the 3x3x3 cube (w = 1 / distance), read from the maps
 * of the previous iteration.  d_params [3][nz][ny][nx] and d_lambda [nz][ny][nx] are updated. */
int kcs_lm_fit(const kcs_geometry* g, const kcs_frames* f, const kcs_kinetics* k, const kcs_prior* p,
               const kcs_lm_opts* lm, const float* d_x, float* d_params, float* d_lambda, void* d_work,
               size_t work_bytes, hipStream_t stream);

/* Initial ICM state: x_m = max(sum_d (s_dm - r_m), 1) / (E_m sum_v sum_d p_vd) in every voxel,
 * maps = xi0 everywhere (n_maps = 3 values K1, k2, k3, or 4 with the blood fraction for studies
 * with kcs_kinetics.fit_vb; d_params is [n_maps][nz][ny][nx]), lambda = 0 (initialised by the
 * first LM iteration).  The flat start ignores g->d_mult (the first OSL update rescales the
 * image to the data). */
int kcs_init_state(const kcs_geometry* g, const kcs_frames* f, const float* d_sino, const double* xi0,
                   int32_t n_maps, float* d_x, float* d_params, float* d_lambda, void* d_work, size_t work_bytes,
                   hipStream_t stream);

/* One ICM sweep (Sec. II-D): kcs_osl_update for q = 0..Q-1 (prior on iff p->kp_on and
 * sweep_idx > 0), then the lm->n_iter iterations of kcs_lm_fit.  With lm->restart the fit starts
 * from tau * max diag(J^T J) whatever d_lambda holds on entry; without it from d_lambda (lambda <= 0
 * initialises).  d_lambda returns the damping after the last iteration. */
int kcs_icm_sweep(const kcs_geometry* g, const kcs_frames* f, const kcs_kinetics* k, const kcs_prior* p,
                  const kcs_lm_opts* lm, const float* d_sino, int32_t Q, int32_t sweep_idx, float* d_x,
                  float* d_params, float* d_lambda, void* d_work, size_t work_bytes, hipStream_t stream);

/* kcs_icm_sweep without a caller workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc).  The workspace
 * is a static array of the library, 256 MiB per GPU, held from the library's load until the
 * process ends; the call itself allocates nothing.  Arguments, results and errors are those of
 * kcs_icm_sweep, plus KCS_EWORKSPACE (nothing launched) when kcs_workspace_bytes(g, M, Q)
 * exceeds 256 MiB (for example 128 x 128 images with M = 24, Q = 6 and more than about 35
 * planes).  All calls on one GPU share that GPU's array: calls that overlap on one GPU (other
 * streams, other host threads) race and must be ordered by the caller.  Nothing in the array
 * carries over from one call to the next. */
int kcs_icm_sweep_noalloc(const kcs_geometry* g, const kcs_frames* f, const kcs_kinetics* k, const kcs_prior* p,
                          const kcs_lm_opts* lm, const float* d_sino, int32_t Q, int32_t sweep_idx, float* d_x,
                          float* d_params, float* d_lambda, hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Batched execution.  A plan runs ICM sweeps of many independent studies (uneven sizes, subset
 * counts and schedules) together: every phase of a sweep (model pass, forward projection,
 * OSL update of subset slot q, map copy, MAP-LM iteration i) is one kernel launch over the
 * concatenated work lists of all studies that take part in it, so small studies fill the GPU
 * together.  Studies are independent: each result equals the single-study calls on the same
 * study up to the projector variant chosen for it (rounding-level differences).
 *
 * kcs_study holds one study's arguments as for kcs_icm_sweep: sweeps sweep_begin..sweep_end-1
 * are run (sweep 0 has the kinetics-derived prior off); d_work is that study's own workspace of
 * kcs_workspace_bytes(&g, M, Q) bytes.  Host arrays in f are only read by kcs_plan_create.
 * ------------------------------------------------------------------------------------------- */
typedef struct kcs_study {
    kcs_geometry g;
    kcs_frames f;
    kcs_kinetics k;
    kcs_prior p;
    kcs_lm_opts lm;
    int32_t Q, sweep_begin, sweep_end;
    const float* d_sino;
    float* d_x;
    float* d_params;
    float* d_lambda;
    void* d_work;
    size_t work_bytes;
} kcs_study;

typedef struct kcs_plan kcs_plan;

enum {
    KCS_PLAN_GRAPH = 1,   /* capture the whole schedule in one HIP graph; kcs_plan_run launches it */
    KCS_PLAN_AUTOTUNE = 2 /* time the projector variants (ray-driven, 16, 32 or 64 pixel tiles) on these
                             studies for every study shape (grid, bins, subset size, frames, pixel/bin
                             ratio) not tuned yet, and keep the fastest for that shape for the rest of
                             the process: every later call on a study of that shape, plain or planned,
                             uses it, so a study's result depends on its shape and not on the call.
                             With KCS_TUNE_CACHE set, tuned shapes are appended to that file and read
                             back by later processes (which then start from them).  It also times one
                             MAP-LM iteration with voxel tiles 64, 32, 16 and 8 voxels wide for every
                             plane shape not tuned yet (writing only workspace regions) and keeps the
                             fastest for the process; the tile changes no result.  The environment
                             variables KCS_PROJ_TILE (0 = ray-driven, 16, 32, 64) and KCS_LM_TILE (8,
                             16, 32, 64), read at every call, override the projector variant and the
                             fit's voxel tile of every study (for measurements and tests) */
};

/* Validates every study (on failure: KCS_EINVAL / KCS_EWORKSPACE naming the study, nothing is
 * launched), enqueues the per-study constant tables (in each workspace) and the upload of the job
 * tables (library-owned device memory) on `stream` without waiting for them, and optionally
 * autotunes (this waits for `stream`) and captures.  The studies' device buffers must stay valid
 * and keep their roles until kcs_plan_destroy; a plan may be run any number of times, and each
 * run repeats the same sweeps (the prior is on for sweep indices above 0). */
int kcs_plan_create(const kcs_study* studies, int32_t n, int32_t flags, hipStream_t stream, kcs_plan** out);

/* Enqueues the whole schedule of the plan on `stream` (asynchronous; ordered after the plan's
 * creation work when that went to another stream).  Runs of plans that share a study must not
 * overlap. */
int kcs_plan_run(kcs_plan* plan, hipStream_t stream);

/* Writes a one-line summary (studies, launches, graph, projector variant per study) into buf. */
int kcs_plan_describe(const kcs_plan* plan, char* buf, size_t len);

/* Waits for the plan's last run and its creation work, then frees its device memory, staging
 * buffer and graph.  NULL is ignored. */
void kcs_plan_destroy(kcs_plan* plan);

/* Kernel timing for measurement harnesses.  While enabled, every kernel or copy the library
 * launches is bracketed by a pair of HIP events recorded on the call's stream (the events are
 * created by the library and reused).  kcs_timing_collect waits for the recorded events, adds
 * the elapsed milliseconds per kind into total_ms[k] and the launch count into count[k]
 * (arrays of KCS_TIMING_KINDS entries, overwritten), and forgets them.  Kinds: */
enum {
    KCS_T_SETUP = 0,   /* table setup */
    KCS_T_PROJECT = 1, /* forward projection (K-proj, with or without the ratio) */
    KCS_T_BACK = 2,    /* plain back projection */
    KCS_T_OSL = 3,     /* back projection fused with the OSL update (K-back) */
    KCS_T_LM = 4,      /* MAP-LM iteration (K-lm) */
    KCS_T_MODEL = 5,   /* model TAC evaluation */
    KCS_T_INIT = 6,    /* initial state */
    KCS_T_COPY = 7,    /* device-to-device copy of the kinetic maps */
    KCS_TIMING_KINDS = 8
};
int kcs_timing_enable(int32_t on);
int kcs_timing_collect(double* total_ms, int64_t* count);

/* Device bandwidth probe for measurement harnesses (no part of the method): kind 0 reads `bytes`
 * from d_src (16-byte aligned, bytes a positive multiple of 16) with a grid-stride loop of
 * `groups` workgroups of 256 threads and writes one partial sum per thread into d_dst
 * (groups * 256 floats); kind 1 copies `bytes` from d_src to d_dst (16-byte aligned, not
 * overlapping).  1 <= groups <= 2^20.  Asynchronous on `stream`; KCS_EINVAL otherwise. */
int kcs_stream_probe(int32_t kind, const void* d_src, void* d_dst, size_t bytes, int32_t groups, hipStream_t stream);

/* Message describing the last error on the calling thread ("" if none). */
const char* kcs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KCS_H */
