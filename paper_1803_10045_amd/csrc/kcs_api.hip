// Host side of libkcs: argument validation, FP64 constants, workspace layout and the C ABI.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "kcs_device.h"
#include "kcs_launch.h"

namespace kcs {
namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(KCS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_finite(double v) { return std::isfinite(v); }

constexpr int32_t kInitChunks = 2048;

// ----------------------------------------------------------------------------------------------
// Validation
int check_geometry(const kcs_geometry* g) {
    if (!g) return fail(KCS_EINVAL, "geometry is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(KCS_EINVAL, "image size must be >= 1");
    if (g->n_ang < 1 || g->n_bin < 1) return fail(KCS_EINVAL, "sinogram size must be >= 1");
    if (!(g->pixel_mm > 0) || !is_finite(g->pixel_mm)) return fail(KCS_EINVAL, "pixel_mm must be > 0");
    if (!(g->bin_mm > 0) || !is_finite(g->bin_mm)) return fail(KCS_EINVAL, "bin_mm must be > 0");
    if (!is_finite(g->ang0_rad)) return fail(KCS_EINVAL, "ang0_rad must be finite");
    if ((double)g->nx * g->ny * g->nz >= 2147483647.0) return fail(KCS_ESHAPE, "more than 2^31 voxels");
    if (g->nx > 16384 || g->ny > 16384 || g->n_bin > 65536) return fail(KCS_ESHAPE, "grid too large");
    return KCS_OK;
}

// A frame that starts within rounding of the previous frame's end (a schedule built as end -
// duration) starts exactly there: such frames share a boundary, whose integrals the model
// evaluates once.
constexpr double kFrameSnap = 1e-12;

bool starts_at_previous_end(const kcs_frames& f, int m) {
    return m > 0 && std::fabs(f.t0_min[m] - f.t1_min[m - 1]) <= kFrameSnap * std::max(1.0, f.t1_min[m - 1]);
}

double frame_start(const kcs_frames& f, int m) { return starts_at_previous_end(f, m) ? f.t1_min[m - 1] : f.t0_min[m]; }

int check_frames(const kcs_frames* f) {
    if (!f) return fail(KCS_EINVAL, "frames is NULL");
    const int M = f->n_frames;
    if (M != 8 && M != 16 && M != 24 && M != 32) return fail(KCS_ESHAPE, "n_frames must be 8, 16, 24 or 32 (got %d)", M);
    if (!f->t0_min || !f->t1_min || !f->scale || !f->bg) return fail(KCS_EINVAL, "frame arrays must not be NULL");
    for (int m = 0; m < M; ++m) {
        if (!is_finite(f->t0_min[m]) || !is_finite(f->t1_min[m]) || f->t0_min[m] < 0 || !(f->t1_min[m] > f->t0_min[m]))
            return fail(KCS_EINVAL, "frame %d: need 0 <= t0 < t1", m);
        if (m > 0 && f->t0_min[m] < f->t1_min[m - 1] && !starts_at_previous_end(*f, m))
            return fail(KCS_EINVAL, "frames must be sorted and disjoint");
        if (!(f->scale[m] > 0) || !is_finite(f->scale[m])) return fail(KCS_EINVAL, "frame %d: scale must be > 0", m);
        if (!(f->bg[m] >= 0) || !is_finite(f->bg[m])) return fail(KCS_EINVAL, "frame %d: bg must be >= 0", m);
    }
    return KCS_OK;
}

int check_kinetics(const kcs_kinetics* k) {
    if (!k) return fail(KCS_EINVAL, "kinetics is NULL");
    const double v[] = {k->A1, k->A2, k->A3, k->l1, k->l2, k->l3, k->vb};
    for (double x : v)
        if (!is_finite(x)) return fail(KCS_EINVAL, "kinetics must be finite");
    if (!(k->l1 < 0 && k->l2 < 0 && k->l3 < 0)) return fail(KCS_EINVAL, "input-function exponents must be negative");
    if (k->fit_vb != 0 && k->fit_vb != 1) return fail(KCS_EINVAL, "fit_vb must be 0 or 1");
    if (!k->fit_vb && !(k->vb >= 0 && k->vb < 1)) return fail(KCS_EINVAL, "vb must be in [0, 1)");
    return KCS_OK;
}

// Number of kinetic maps of a study: K1, k2, k3 and, with fit_vb, the blood fraction.
int n_maps(const kcs_kinetics& k) { return k.fit_vb ? 4 : 3; }

int check_prior(const kcs_prior* p, int np = 3) {
    if (!p) return fail(KCS_EINVAL, "prior is NULL");
    if (!(p->beta_kp >= 0 && p->beta_kp < 1)) return fail(KCS_EINVAL, "beta_kp must be in [0, 1)");
    if (!(p->eps_F > 0) || !is_finite(p->eps_F)) return fail(KCS_EINVAL, "eps_F must be > 0");
    if (!(p->beta_h >= 0) || !is_finite(p->beta_h)) return fail(KCS_EINVAL, "beta_h must be >= 0");
    for (int i = 0; i < np; ++i)
        if (!(p->delta[i] > 0) || !is_finite(p->delta[i])) return fail(KCS_EINVAL, "delta must be > 0");
    if (!(p->plane_ratio >= 0) || !is_finite(p->plane_ratio)) return fail(KCS_EINVAL, "plane_ratio must be >= 0");
    return KCS_OK;
}

int check_lm(const kcs_lm_opts* o, int np = 3) {
    if (!o) return fail(KCS_EINVAL, "lm options are NULL");
    if (o->n_iter < 0 || o->n_iter > 100000) return fail(KCS_EINVAL, "n_iter out of range");
    if (!(o->tau > 0) || !(o->lam_min > 0) || !(o->lam_max >= o->lam_min) || !is_finite(o->lam_max))
        return fail(KCS_EINVAL, "need tau > 0 and 0 < lam_min <= lam_max");
    for (int i = 0; i < np; ++i)
        if (!is_finite(o->lo[i]) || !is_finite(o->hi[i]) || !(o->lo[i] <= o->hi[i])) return fail(KCS_EINVAL, "need lo <= hi");
    if (np == 4 && !(o->lo[3] >= 0 && o->hi[3] <= 1)) return fail(KCS_EINVAL, "blood fraction bounds must lie in [0, 1]");
    if (!(o->lo[1] + o->lo[2] > 0)) return fail(KCS_EINVAL, "lo[1] + lo[2] must be > 0 (k2 + k3 > 0)");
    if (!(o->eta >= 0 && o->eta < 1)) return fail(KCS_EINVAL, "eta must be in [0, 1)");
    return KCS_OK;
}

// Offsets within one plane's image (j * nx * M + i * M) are 32-bit in the kernels.
int check_plane(const kcs_geometry* g, int32_t M) {
    if ((double)g->nx * g->ny * M >= 2147483647.0) return fail(KCS_ESHAPE, "a plane of nx*ny*M >= 2^31 values");
    return KCS_OK;
}

int check_subset(const kcs_geometry* g, int32_t q, int32_t Q) {
    if (Q < 1 || Q > g->n_ang) return fail(KCS_EINVAL, "need 1 <= Q <= n_ang");
    if (q < 0 || q >= Q) return fail(KCS_EINVAL, "need 0 <= q < Q");
    if ((g->n_ang + Q - 1) / Q > 1024) return fail(KCS_ESHAPE, "more than 1024 angles in a subset");
    if (!staged_fits(kMaxFrames, (float)g->pixel_mm, (float)g->bin_mm))
        return fail(KCS_ESHAPE, "bins more than 6 times narrower than pixels are not supported");
    return KCS_OK;
}

#define KCS_TRY(x)                  \
    do {                            \
        const int _rc = (x);        \
        if (_rc != KCS_OK) return _rc; \
    } while (0)

// ----------------------------------------------------------------------------------------------
// FP64 constants

// m_k(x) = int_0^1 s^k e^{x s} ds, k = 0..2, for x <= 0 (series near 0, recursion otherwise)
void moments3(double x, double m[3]) {
    if (std::fabs(x) < 1.0) {
        double term = 1.0;
        m[0] = m[1] = m[2] = 0.0;
        for (int j = 0; j < 30; ++j) {
            for (int k = 0; k < 3; ++k) m[k] += term / (j + k + 1);
            term *= x / (j + 1);
        }
        return;
    }
    const double e = std::exp(x);
    m[0] = std::expm1(x) / x;
    m[1] = (e - m[0]) / x;
    m[2] = (e - 2.0 * m[1]) / x;
}

// P1(t) = int_0^t Cp and P2(t) = int_0^t P1 for the Feng input (sum of c t^n e^{l t} terms)
void input_integrals(const kcs_kinetics& k, double t, double& P1, double& P2) {
    const double c[4] = {k.A1, -(k.A2 + k.A3), k.A2, k.A3};
    const double l[4] = {k.l1, k.l1, k.l2, k.l3};
    const int n[4] = {1, 0, 0, 0};
    P1 = P2 = 0.0;
    for (int i = 0; i < 4; ++i) {
        double m[3];
        moments3(l[i] * t, m);
        const double tp = std::pow(t, n[i] + 1);
        P1 += c[i] * tp * m[n[i]];
        P2 += c[i] * tp * t * (m[n[i]] - m[n[i] + 1]);
    }
}

struct Schedule {
    FrameTab fr;
    SetupArgs setup;
};

Schedule make_schedule(const kcs_frames& f, const kcs_kinetics* k) {
    Schedule S{};
    const int M = f.n_frames;
    S.fr.M = M;
    S.fr.contiguous = 1;
    for (int m = 1; m < M; ++m)
        if (frame_start(f, m) != f.t1_min[m - 1]) S.fr.contiguous = 0;
    std::vector<double> tb;
    for (int m = 0; m < M; ++m) {
        tb.push_back(frame_start(f, m));
        tb.push_back(f.t1_min[m]);
    }
    std::sort(tb.begin(), tb.end());
    tb.erase(std::unique(tb.begin(), tb.end()), tb.end());
    S.setup.n_bound = (int32_t)tb.size();
    for (size_t b = 0; b < tb.size(); ++b) S.setup.t[b] = tb[b];
    S.setup.M = M;
    for (int m = 0; m < M; ++m) {
        S.setup.i0[m] = (int32_t)(std::lower_bound(tb.begin(), tb.end(), frame_start(f, m)) - tb.begin());
        S.setup.i1[m] = (int32_t)(std::lower_bound(tb.begin(), tb.end(), f.t1_min[m]) - tb.begin());
        const double dt = f.t1_min[m] - frame_start(f, m);
        S.fr.E[m] = (float)f.scale[m];
        S.fr.r[m] = (float)f.bg[m];
        S.fr.inv_dt[m] = (float)(1.0 / dt);
    }
    if (k) {
        S.setup.A1 = k->A1;
        S.setup.A2 = k->A2;
        S.setup.A3 = k->A3;
        S.setup.l[0] = k->l1;
        S.setup.l[1] = k->l2;
        S.setup.l[2] = k->l3;
        S.setup.vb = k->vb;
        S.fr.one_minus_vb = (float)(1.0 - k->vb);
        for (int m = 0; m < M; ++m) {
            double a1, a2, b1, b2;
            input_integrals(*k, frame_start(f, m), a1, a2);
            input_integrals(*k, f.t1_min[m], b1, b2);
            S.fr.blood[m] = (float)(k->vb * (b1 - a1));
            S.fr.cp_int[m] = (float)(b1 - a1);
            S.fr.dP2[m] = (float)(b2 - a2);
        }
    }
    return S;
}

int32_t subset_size(const kcs_geometry& g, int32_t q, int32_t Q) { return (g.n_ang - q + Q - 1) / Q; }

ProjArgs proj_args(const kcs_geometry& g, const FrameTab& fr, int32_t q, int32_t Q) {
    ProjArgs p{};
    p.nx = g.nx;
    p.ny = g.ny;
    p.nz = g.nz;
    p.n_ang = g.n_ang;
    p.n_bin = g.n_bin;
    p.q = q;
    p.Q = Q;
    p.A_q = subset_size(g, q, Q);
    p.rays_per_plane = p.A_q * g.n_bin;
    p.h = (float)g.pixel_mm;
    p.inv_h = (float)(1.0 / g.pixel_mm);
    p.du = (float)g.bin_mm;
    p.inv_du = (float)(1.0 / g.bin_mm);
    p.ang0 = g.ang0_rad;
    p.hd = g.pixel_mm;
    p.dud = g.bin_mm;
    p.mult = g.d_mult;
    p.fr = fr;
    return p;
}

// Total length of all rays inside the image square: sum_v sum_d p_vd over one plane.
double total_path_length(const kcs_geometry& g) {
    const double h = g.pixel_mm, X0 = -0.5 * g.nx * h, Y0 = -0.5 * g.ny * h;
    double tot = 0.0;
    for (int a = 0; a < g.n_ang; ++a) {
        const double th = g.ang0_rad + (double)a * 3.141592653589793 / (double)g.n_ang;
        double c = std::cos(th), s = std::sin(th);
        if (std::fabs(c) < 1e-12) {
            c = 0.0;
            s = s > 0 ? 1.0 : -1.0;
        }
        if (std::fabs(s) < 1e-12) {
            s = 0.0;
            c = c > 0 ? 1.0 : -1.0;
        }
        for (int b = 0; b < g.n_bin; ++b) {
            const double u = ((double)b - 0.5 * (g.n_bin - 1)) * g.bin_mm;
            // clip the line {u (c, s) + t (-s, c)} to the half-open rectangle
            double t0 = -1e300, t1 = 1e300;
            const double px = u * c, py = u * s, dx = -s, dy = c;
            bool miss = false;
            auto clip = [&](double p0, double d, double lo, double hi) {
                if (d == 0.0) {
                    if (!(p0 >= lo && p0 < hi)) miss = true;
                    return;
                }
                double a0 = (lo - p0) / d, a1 = (hi - p0) / d;
                if (a0 > a1) std::swap(a0, a1);
                t0 = std::max(t0, a0);
                t1 = std::min(t1, a1);
            };
            clip(px, dx, X0, -X0);
            clip(py, dy, Y0, -Y0);
            if (!miss && t1 > t0) tot += t1 - t0;
        }
    }
    return tot;
}

// Workspace layout
struct Layout {
    size_t kin, xi, lms, init, F, ratio, psum, total;
};

// ----- forward projector variant per shape -----
// The variants (ray-driven, LDS tiles of 16, 32 or 64 pixels) add a ray's line integral in
// different orders, so they round differently.  A study's variant is a function of its shape
// only, the same for plain calls and plans: the default rule below, or the variant the plan
// autotuner measured for that shape, which it records here for the rest of the process (and in
// the file named by KCS_TUNE_CACHE, from which later processes start).
struct TuneKey {
    int nx, ny, n_bin, A_q, M;
    float hdu;
    bool operator==(const TuneKey& o) const {
        return nx == o.nx && ny == o.ny && n_bin == o.n_bin && A_q == o.A_q && M == o.M && hdu == o.hdu;
    }
};

TuneKey tune_key(const kcs_geometry& g, int M, int32_t Q) {
    return TuneKey{g.nx, g.ny, g.n_bin, (g.n_ang + Q - 1) / Q, M, (float)(g.pixel_mm / g.bin_mm)};
}

std::recursive_mutex g_tune_mu;  // recursive: the tuner builds job arguments that look tuned values up
std::vector<std::pair<TuneKey, int>> g_tuned;  // guarded by g_tune_mu
bool g_tune_file_read = false;

// Tuned variant of a shape, or -1; on first use loads the KCS_TUNE_CACHE file.  Caller holds
// g_tune_mu.
int tuned_tile_locked(const TuneKey& k) {
    if (!g_tune_file_read) {
        g_tune_file_read = true;
        const char* path = getenv("KCS_TUNE_CACHE");
        if (FILE* f = path ? fopen(path, "r") : nullptr) {
            int nx, ny, nb, aq, M, T;
            float hdu, ms;
            while (fscanf(f, "%d %d %d %d %d %f %d %f", &nx, &ny, &nb, &aq, &M, &hdu, &T, &ms) == 8) {
                if (T != 0 && T != 16 && T != 32 && T != 64) continue;
                const TuneKey key{nx, ny, nb, aq, M, hdu};
                bool seen = false;
                for (auto& e : g_tuned)
                    if (e.first == key) {
                        e.second = T;  // the file's last entry for a shape wins
                        seen = true;
                    }
                if (!seen) g_tuned.push_back({key, T});
            }
            fclose(f);
        }
    }
    for (const auto& e : g_tuned)
        if (e.first == k) return e.second;
    return -1;
}

// Voxel tile width of the MAP-LM kernel for a plane shape: KCS_LM_TILE (8, 16, 32, 64)
// overrides; then the width the plan autotuner measured fastest for that shape in this process,
// otherwise lm_tile_x's rule.  The tile does not change any voxel's result.
std::vector<std::pair<std::pair<int, int>, int>> g_lm_tile;  // (nx, ny) -> tile width; guarded by g_tune_mu

int lm_tile_for(int nx, int ny) {
    if (const char* e = getenv("KCS_LM_TILE")) {
        const int t = atoi(e);
        if (t == 8 || t == 16 || t == 32 || t == 64) return t;
    }
    std::lock_guard<std::recursive_mutex> lk(g_tune_mu);
    for (const auto& e : g_lm_tile)
        if (e.first == std::make_pair(nx, ny)) return e.second;
    return lm_tile_x(nx, ny);
}

// Variant for a study shape: KCS_PROJ_TILE (0, 16, 32, 64) overrides; then a tuned variant of
// this shape; otherwise LDS tiles of 32 pixels for planes beyond an XCD's L2 share (2 MB),
// ray-driven below.
int projector_tile(const kcs_geometry& g, int M, int32_t Q) {
    if (const char* e = getenv("KCS_PROJ_TILE")) {
        const int t = atoi(e);
        if (t == 0 || t == 16 || t == 32 || t == 64) return t;
    }
    {
        std::lock_guard<std::recursive_mutex> lk(g_tune_mu);
        const int t = tuned_tile_locked(tune_key(g, M, Q));
        if (t >= 0) return t;
    }
    const double plane_bytes = (double)g.nx * g.ny * M * 4.0;
    return plane_bytes < 2.0 * 1024 * 1024 ? 0 : 32;
}

// Offsets of the workspace regions.  The model TACs of the maps and the ratio buffer (the
// largest subset's sinogram) come last so that calls without projections (Q = 0) need only the
// leading regions.
Layout layout(const kcs_geometry* g, int32_t M, int32_t Q) {
    Layout L{};
    size_t off = 0;
    L.kin = off;
    off = align_up(off + sizeof(KinTab), 256);
    if (g) {
        const size_t N = (size_t)g->nx * g->ny * g->nz;
        L.xi = off;
        off = align_up(off + 4 * N * sizeof(float), 256);  // up to 4 maps (with the blood fraction)
        L.lms = off;  // MAP-LM normal equations carried between iterations: 10 (15 with 4 maps) floats per voxel
        off = align_up(off + 15 * N * sizeof(float), 256);
        L.init = off;
        off = align_up(off + ((size_t)kInitChunks * M + M) * sizeof(double), 256);
        L.F = off;
        if (Q > 0) off = align_up(off + N * M * sizeof(float), 256);
        L.ratio = off;
        L.psum = off;
        if (Q > 0) {
            const size_t A_max = (size_t)((g->n_ang + Q - 1) / Q);
            off = align_up(off + (size_t)g->nz * A_max * g->n_bin * M * sizeof(float), 256);
            L.psum = off;
            ProjArgs pa{};
            pa.nx = g->nx;
            pa.ny = g->ny;
            pa.nz = g->nz;
            pa.A_q = (int32_t)A_max;
            pa.h = (float)g->pixel_mm;
            pa.du = (float)g->bin_mm;
            off = align_up(off + std::max({tile_partial_bytes(16, pa, M), tile_partial_bytes(32, pa, M),
                                           tile_partial_bytes(64, pa, M)}),
                           256);
        }
    }
    L.total = off;
    return L;
}

int check_work(const kcs_geometry* g, int32_t M, int32_t Q, void* d_work, size_t work_bytes) {
    if (!d_work) return fail(KCS_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(d_work) & 255) != 0) return fail(KCS_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = layout(g, M, Q).total;
    if (work_bytes < need) return fail(KCS_EWORKSPACE, "workspace has %zu bytes, needs %zu", work_bytes, need);
    return KCS_OK;
}

template <class T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

int launched(hipError_t e, const char* what) { return e == hipSuccess ? KCS_OK : hip_fail(e, what); }

// Optional event timing of every launch (measurement only).
struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimedLaunch> g_launches;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t pooled_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs `launch` (which enqueues work on `st`), bracketed by events when timing is enabled.
template <class F>
hipError_t timed(int kind, hipStream_t st, F&& launch) {
    std::unique_lock<std::mutex> lk(g_tmu);
    if (!g_timing) {
        lk.unlock();
        return launch();
    }
    hipEvent_t a = pooled_event(), b = pooled_event();
    if (a) hipEventRecord(a, st);
    const hipError_t e = launch();
    if (b) hipEventRecord(b, st);
    if (a && b) g_launches.push_back({kind, a, b});
    return e;
}

// Internal bodies (arguments already validated)
int do_setup(const Schedule& S, void* d_work, hipStream_t st) {
    return launched(timed(KCS_T_SETUP, st, [&] { return launch_setup(S.setup, at<KinTab>(d_work, layout(nullptr, 0, 0).kin), st); }),
                    "table setup");
}

// Model TACs of the maps into the workspace (read by every OSL update of the pass).
int do_model_pass(const kcs_geometry& g, const Schedule& S, int np, const float* params, void* d_work, int32_t Q,
                  hipStream_t st) {
    const Layout L = layout(&g, S.fr.M, Q);
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    return launched(timed(KCS_T_MODEL, st,
                          [&] {
                              return launch_model(S.fr.M, np, at<KinTab>(d_work, L.kin), S.fr, params, N,
                                                  at<float>(d_work, L.F), nullptr, st);
                          }),
                    "model pass");
}

int do_osl(const kcs_geometry& g, const Schedule& S, const kcs_prior& p, bool kp, const float* sino, int32_t q,
           int32_t Q, float* x, void* d_work, hipStream_t st) {
    const Layout L = layout(&g, S.fr.M, Q);
    OslArgs a{};
    a.g = proj_args(g, S.fr, q, Q);
    a.beta_kp = (float)p.beta_kp;
    a.eps_F = (float)p.eps_F;
    a.kp = kp ? 1 : 0;
    float* ratio = at<float>(d_work, L.ratio);
    const int T = projector_tile(g, S.fr.M, Q);
    float* psum = at<float>(d_work, L.psum);
    KCS_TRY(launched(timed(KCS_T_PROJECT, st,
                           [&] {
                               return T ? launch_project_tiled(S.fr.M, T, x, sino, ratio, psum, a.g, true, st)
                                        : launch_project(S.fr.M, x, sino, ratio, a.g, true, st);
                           }),
                     "forward projection"));
    const float* Fm = at<float>(d_work, L.F);
    return launched(timed(KCS_T_OSL, st, [&] { return launch_osl(S.fr.M, ratio, Fm, x, a, st); }), "OSL update");
}

// Neighbourhood of the Huber term: in-plane 3x3, or the 3x3x3 cube with planes plane_ratio
// pixel sides apart, each neighbour weighted by 1 / its distance.
void set_neighbourhood(LmArgs& a, const kcs_prior& p) {
    a.nbr3d = p.plane_ratio > 0 ? 1 : 0;
    const double r2 = p.plane_ratio * p.plane_ratio;
    for (int k = 0; k < 3; ++k) a.w_plane[k] = a.nbr3d ? (float)(1.0 / std::sqrt(r2 + k)) : 0.0f;
}

int do_lm(const kcs_geometry& g, const Schedule& S, int np, const kcs_prior& p, const kcs_lm_opts& o, const float* x,
          float* params, float* lam, void* d_work, int32_t Q, bool fresh_lambda, hipStream_t st) {
    if (o.n_iter == 0) return KCS_OK;
    const Layout L = layout(&g, S.fr.M, Q);
    const size_t N = (size_t)g.nx * g.ny * g.nz;
    LmArgs a{};
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.tile_x = lm_tile_for(g.nx, g.ny);
    a.fr = S.fr;
    a.beta_h = (float)p.beta_h;
    set_neighbourhood(a, p);
    a.np = np;
    for (int i = 0; i < np; ++i) {
        a.delta[i] = (float)p.delta[i];
        a.lo[i] = (float)o.lo[i];
        a.hi[i] = (float)o.hi[i];
    }
    a.tau = (float)o.tau;
    a.eta = (float)o.eta;
    a.lam_min = (float)o.lam_min;
    a.lam_max = (float)o.lam_max;
    float* other = at<float>(d_work, L.xi);
    // ping-pong so that the last iteration writes into `params`
    float* src = params;
    float* dst = other;
    if (o.n_iter % 2 == 1) {
        hipError_t e = timed(KCS_T_COPY, st, [&] {
            return hipMemcpyAsync(other, params, np * N * sizeof(float), hipMemcpyDeviceToDevice, st);
        });
        if (e != hipSuccess) return hip_fail(e, "map copy");
        src = other;
        dst = params;
    }
    const KinTab* K = at<KinTab>(d_work, L.kin);
    float* state = at<float>(d_work, L.lms);
    for (int it = 0; it < o.n_iter; ++it) {
        a.reset_lambda = (fresh_lambda && it == 0) ? 1 : 0;
        a.have_state = it > 0 ? 1 : 0;
        a.need_state = it + 1 < o.n_iter ? 1 : 0;
        KCS_TRY(launched(timed(KCS_T_LM, st, [&] { return launch_lm(S.fr.M, K, x, src, dst, lam, state, a, st); }),
                         "MAP-LM iteration"));
        std::swap(src, dst);
    }
    return KCS_OK;
}


// ---------------------------------------------------------------------------------------------
// Batched plans

enum PhaseKind { PH_MODEL, PH_PROJ, PH_REDUCE, PH_OSL, PH_COPY, PH_LM };

struct PlanPhase {
    int kind, M, T;
    size_t off;         // byte offset of the job table in the plan's device buffer
    size_t starts_off;  // byte offset of the packed first-workgroup indices of the jobs
    int n;              // jobs
    uint32_t groups;
    int max_angles;
};

struct StudyPrep {
    const kcs_study* s;
    Schedule S;
    Layout L;
    int T;  // forward projector variant
};

// Host image of the job tables: phases append their jobs (w0 = running work index).
struct TableBuilder {
    std::vector<char> buf;
    std::vector<PlanPhase> phases;

    template <class Job>
    void add(int kind, int M, int T, std::vector<Job>& jobs, const std::vector<uint32_t>& groups, int max_angles) {
        if (jobs.empty()) return;
        uint32_t w = 0;
        for (size_t k = 0; k < jobs.size(); ++k) {
            jobs[k].w0 = w;
            w += groups[k];
        }
        const size_t soff = align_up(buf.size(), 256);
        const size_t off = align_up(soff + jobs.size() * sizeof(uint32_t), 256);
        buf.resize(off + jobs.size() * sizeof(Job));
        for (size_t k = 0; k < jobs.size(); ++k) memcpy(buf.data() + soff + 4 * k, &jobs[k].w0, 4);
        memcpy(buf.data() + off, jobs.data(), jobs.size() * sizeof(Job));
        phases.push_back(PlanPhase{kind, M, T, off, soff, (int)jobs.size(), w, max_angles});
    }
};

int check_study(const kcs_study& st) {
    KCS_TRY(check_geometry(&st.g));
    KCS_TRY(check_frames(&st.f));
    KCS_TRY(check_plane(&st.g, st.f.n_frames));
    KCS_TRY(check_kinetics(&st.k));
    if (st.k.fit_vb) return fail(KCS_EINVAL, "plans do not fit the blood fraction (fit_vb)");
    KCS_TRY(check_prior(&st.p));
    KCS_TRY(check_lm(&st.lm));
    KCS_TRY(check_subset(&st.g, 0, st.Q));
    if (st.sweep_begin < 0 || st.sweep_end < st.sweep_begin) return fail(KCS_EINVAL, "need 0 <= sweep_begin <= sweep_end");
    if (!st.d_sino || !st.d_x || !st.d_params || !st.d_lambda) return fail(KCS_EINVAL, "study pointers must not be NULL");
    return check_work(&st.g, st.f.n_frames, st.Q, st.d_work, st.work_bytes);
}

ProjJob proj_job(const StudyPrep& P, int q) {
    const kcs_study& s = *P.s;
    ProjJob j{};
    j.p = proj_args(s.g, P.S.fr, q, s.Q);
    j.x = s.d_x;
    j.sino = s.d_sino;
    j.out = at<float>(s.d_work, P.L.ratio);
    j.psum = at<float>(s.d_work, P.L.psum);
    j.slots = P.T ? tile_slots(P.T, j.p.h, j.p.du) : 0;
    return j;
}

LmArgs lm_args(const StudyPrep& P) {
    const kcs_study& s = *P.s;
    LmArgs a{};
    a.nx = s.g.nx;
    a.ny = s.g.ny;
    a.nz = s.g.nz;
    a.tile_x = lm_tile_for(s.g.nx, s.g.ny);
    a.fr = P.S.fr;
    a.beta_h = (float)s.p.beta_h;
    set_neighbourhood(a, s.p);
    a.np = 3;
    for (int i = 0; i < 3; ++i) {
        a.delta[i] = (float)s.p.delta[i];
        a.lo[i] = (float)s.lm.lo[i];
        a.hi[i] = (float)s.lm.hi[i];
    }
    a.tau = (float)s.lm.tau;
    a.eta = (float)s.lm.eta;
    a.lam_min = (float)s.lm.lam_min;
    a.lam_max = (float)s.lm.lam_max;
    return a;
}

// Forward projections of subset slot q for the studies in `ps` (grouped by frame count and
// projector variant): tile step and reduce step for tiled studies, one launch otherwise.
void add_projection(TableBuilder& tb, const std::vector<const StudyPrep*>& ps, int q) {
    std::vector<std::pair<int, int>> keys;
    for (const StudyPrep* P : ps)
        if (std::find(keys.begin(), keys.end(), std::make_pair(P->S.fr.M, P->T)) == keys.end())
            keys.push_back({P->S.fr.M, P->T});
    for (const auto& key : keys) {
        std::vector<ProjJob> jobs, red;
        std::vector<uint32_t> g, gr;
        int max_a = 1;
        for (const StudyPrep* P : ps) {
            if (P->S.fr.M != key.first || P->T != key.second) continue;
            ProjJob j = proj_job(*P, q);
            max_a = std::max(max_a, (int)j.p.A_q);
            jobs.push_back(j);
            g.push_back(key.second ? proj_tile_groups(j.p, key.second) : proj_direct_groups(j.p));
            red.push_back(j);
            gr.push_back(proj_reduce_groups(j.p));
        }
        tb.add(PH_PROJ, key.first, key.second, jobs, g, max_a);
        if (key.second) tb.add(PH_REDUCE, key.first, key.second, red, gr, max_a);
    }
}

std::vector<int> frame_counts(const std::vector<const StudyPrep*>& ps) {
    std::vector<int> Ms;
    for (const StudyPrep* P : ps)
        if (std::find(Ms.begin(), Ms.end(), P->S.fr.M) == Ms.end()) Ms.push_back(P->S.fr.M);
    return Ms;
}

void build_schedule(TableBuilder& tb, std::vector<StudyPrep>& preps) {
    int s0 = INT32_MAX, s1 = 0;
    for (const StudyPrep& P : preps) {
        if (P.s->sweep_end <= P.s->sweep_begin) continue;
        s0 = std::min(s0, P.s->sweep_begin);
        s1 = std::max(s1, P.s->sweep_end);
    }
    for (int sw = s0; sw < s1; ++sw) {
        std::vector<const StudyPrep*> act;
        for (const StudyPrep& P : preps)
            if (sw >= P.s->sweep_begin && sw < P.s->sweep_end) act.push_back(&P);
        // model TACs of the maps for the studies whose prior is on in this sweep
        for (int M : frame_counts(act)) {
            std::vector<ModelJob> jobs;
            std::vector<uint32_t> g;
            for (const StudyPrep* P : act) {
                if (P->S.fr.M != M || !(P->s->p.kp_on && sw > 0)) continue;
                const kcs_study& s = *P->s;
                const int64_t N = (int64_t)s.g.nx * s.g.ny * s.g.nz;
                jobs.push_back(ModelJob{P->S.fr, at<KinTab>(s.d_work, P->L.kin), s.d_params, N,
                                        at<float>(s.d_work, P->L.F), nullptr, 0});
                g.push_back(model_groups(N));
            }
            tb.add(PH_MODEL, M, 0, jobs, g, 0);
        }
        int qmax = 0;
        for (const StudyPrep* P : act) qmax = std::max(qmax, (int)P->s->Q);
        for (int q = 0; q < qmax; ++q) {
            std::vector<const StudyPrep*> sub;
            for (const StudyPrep* P : act)
                if (q < P->s->Q) sub.push_back(P);
            add_projection(tb, sub, q);
            for (int M : frame_counts(sub)) {
                std::vector<OslJob> jobs;
                std::vector<uint32_t> g;
                int max_a = 1;
                for (const StudyPrep* P : sub) {
                    if (P->S.fr.M != M) continue;
                    const kcs_study& s = *P->s;
                    OslJob j{};
                    j.a.g = proj_args(s.g, P->S.fr, q, s.Q);
                    j.a.beta_kp = (float)s.p.beta_kp;
                    j.a.eps_F = (float)s.p.eps_F;
                    j.a.kp = (s.p.kp_on && sw > 0) ? 1 : 0;
                    j.ratio = at<float>(s.d_work, P->L.ratio);
                    j.Fm = at<float>(s.d_work, P->L.F);
                    j.x = s.d_x;
                    max_a = std::max(max_a, (int)j.a.g.A_q);
                    jobs.push_back(j);
                    g.push_back(staged_tile_groups(s.g.nx, s.g.ny, s.g.nz));
                }
                tb.add(PH_OSL, M, 0, jobs, g, max_a);
            }
        }
        // MAP-LM: maps ping-pong between d_params and the workspace so the last iteration writes
        // d_params; an odd iteration count starts with a copy
        std::vector<CopyJob> cj;
        std::vector<uint32_t> cg;
        int itmax = 0;
        for (const StudyPrep* P : act) {
            itmax = std::max(itmax, (int)P->s->lm.n_iter);
            if (P->s->lm.n_iter % 2 == 1) {
                const kcs_study& s = *P->s;
                const int64_t n3 = 3LL * s.g.nx * s.g.ny * s.g.nz;
                cj.push_back(CopyJob{s.d_params, at<float>(s.d_work, P->L.xi), n3, 0});
                cg.push_back(copy_groups(n3));
            }
        }
        tb.add(PH_COPY, 0, 0, cj, cg, 0);
        for (int it = 0; it < itmax; ++it) {
            for (int M : frame_counts(act)) for (int nb = 0; nb < 2; ++nb) {
                // one launch per frame count and neighbourhood (in-plane / 3x3x3)
                std::vector<LmJob> jobs;
                std::vector<uint32_t> g;
                for (const StudyPrep* P : act) {
                    const kcs_study& s = *P->s;
                    if (P->S.fr.M != M || it >= s.lm.n_iter || (s.p.plane_ratio > 0) != (nb == 1)) continue;
                    float* other = at<float>(s.d_work, P->L.xi);
                    const bool odd = s.lm.n_iter % 2 == 1;
                    const bool even_it = it % 2 == 0;
                    // odd count: it0 other->params, it1 params->other, ...; even: params->other first
                    const float* src = (odd == even_it) ? other : s.d_params;
                    float* dst = (odd == even_it) ? s.d_params : other;
                    LmArgs a = lm_args(*P);
                    a.reset_lambda = (it == 0 && s.lm.restart) ? 1 : 0;
                    a.have_state = it > 0 ? 1 : 0;
                    a.need_state = it + 1 < s.lm.n_iter ? 1 : 0;
                    jobs.push_back(LmJob{a, at<KinTab>(s.d_work, P->L.kin), s.d_x, src, dst, s.d_lambda,
                                         at<float>(s.d_work, P->L.lms), 0});
                    g.push_back(lm_groups(s.g.nx, s.g.ny, s.g.nz, a.tile_x));
                }
                tb.add(PH_LM, M, nb, jobs, g, 0);
            }
        }
    }
}

template <class J>
JobTable<J> table(const PlanPhase& ph, const char* base) {
    return JobTable<J>{reinterpret_cast<const J*>(base + ph.off), reinterpret_cast<const uint32_t*>(base + ph.starts_off),
                       ph.n};
}

hipError_t run_phase(const PlanPhase& ph, const char* base, hipStream_t st) {
    switch (ph.kind) {
        case PH_MODEL: return launch_model_jobs(ph.M, table<ModelJob>(ph, base), ph.groups, st);
        case PH_PROJ:
            return launch_project_jobs(ph.M, ph.T, table<ProjJob>(ph, base), ph.groups, ph.max_angles, true, st);
        case PH_REDUCE: return launch_project_reduce_jobs(ph.M, ph.T, table<ProjJob>(ph, base), ph.groups, true, st);
        case PH_OSL: return launch_osl_jobs(ph.M, table<OslJob>(ph, base), ph.groups, ph.max_angles, st);
        case PH_COPY: return launch_copy_jobs(table<CopyJob>(ph, base), ph.groups, st);
        case PH_LM: return launch_lm_jobs(ph.M, ph.T != 0, table<LmJob>(ph, base), ph.groups, st);
        default: return hipErrorInvalidValue;
    }
}

void store_tile(const TuneKey& k, int T, float ms) {
    const char* path = getenv("KCS_TUNE_CACHE");
    if (!path) return;
    if (FILE* f = fopen(path, "a")) {
        fprintf(f, "%d %d %d %d %d %.6g %d %.6g\n", k.nx, k.ny, k.n_bin, k.A_q, k.M, k.hdu, T, ms);
        fclose(f);
    }
}

// Times one MAP-LM iteration of the studies `cls` (one plane shape) with each voxel tile width
// and keeps the fastest for the shape (caller holds g_tune_mu).  The iteration reads the study's
// image and maps and writes only workspace regions: the maps into the ping-pong buffer, lambda
// into the model-TAC region, the normal equations into their own region.
int tune_lm_tile(const std::vector<StudyPrep*>& cls, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    const kcs_study& s0 = *cls[0]->s;
    const std::pair<int, int> shape{s0.g.nx, s0.g.ny};
    for (const auto& e : g_lm_tile)
        if (e.first == shape) return KCS_OK;
    const int M = s0.f.n_frames;
    const bool nb = s0.p.plane_ratio > 0;
    for (const StudyPrep* P : cls)
        if (P->s->f.n_frames != M || (P->s->p.plane_ratio > 0) != nb) return KCS_OK;  // mixed class: keep the rule
    int best = lm_tile_x(shape.first, shape.second);
    float best_ms = 1e30f;
    for (int tx : {64, 32, 16, 8}) {
        TableBuilder tb;
        std::vector<LmJob> jobs;
        std::vector<uint32_t> g;
        for (const StudyPrep* P : cls) {
            const kcs_study& s = *P->s;
            LmArgs a = lm_args(*P);
            a.tile_x = tx;
            a.reset_lambda = 1;
            a.have_state = 0;
            a.need_state = 0;
            jobs.push_back(LmJob{a, at<KinTab>(s.d_work, P->L.kin), s.d_x, s.d_params, at<float>(s.d_work, P->L.xi),
                                 at<float>(s.d_work, P->L.F), at<float>(s.d_work, P->L.lms), 0});
            g.push_back(lm_groups(s.g.nx, s.g.ny, s.g.nz, tx));
        }
        tb.add(PH_LM, M, nb ? 1 : 0, jobs, g, 0);
        void* dtab = nullptr;
        if (hipMalloc(&dtab, std::max<size_t>(tb.buf.size(), 256)) != hipSuccess) return fail(KCS_EHIP, "tuning table");
        hipError_t e = hipMemcpy(dtab, tb.buf.data(), tb.buf.size(), hipMemcpyHostToDevice);
        float ms = 0.0f;
        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // rep 0 warms up
            if (rep == 1) e = hipEventRecord(e0, st);
            for (const PlanPhase& ph : tb.phases)
                if (e == hipSuccess) e = run_phase(ph, (const char*)dtab, st);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        (void)hipFree(dtab);
        if (e != hipSuccess) return hip_fail(e, "MAP-LM tile tuning");
        if (ms < best_ms) {
            best_ms = ms;
            best = tx;
        }
    }
    g_lm_tile.push_back({shape, best});
    return KCS_OK;
}

// Times the projector variants on the studies of each shape not tuned yet in this process (or in
// the KCS_TUNE_CACHE file), keeps the fastest for the shape (plain calls of that shape use it from
// now on) and appends it to the file.
int autotune(std::vector<StudyPrep>& preps, hipStream_t st) {
    std::lock_guard<std::recursive_mutex> lk(g_tune_mu);
    std::vector<TuneKey> keys;
    for (const StudyPrep& P : preps) {
        const TuneKey k = tune_key(P.s->g, P.s->f.n_frames, P.s->Q);
        if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
    }
    void* dtab = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(KCS_EHIP, "tuning events");
    int rc = KCS_OK;
    for (const TuneKey& k : keys) {
        std::vector<StudyPrep*> cls;
        for (StudyPrep& P : preps)
            if (tune_key(P.s->g, P.s->f.n_frames, P.s->Q) == k) cls.push_back(&P);
        int best = tuned_tile_locked(k);
        if (best < 0) {
            float best_ms = 1e30f;
            for (int T : {0, 16, 32, 64}) {
                for (StudyPrep* P : cls) P->T = T;
                TableBuilder tb;
                std::vector<const StudyPrep*> ps(cls.begin(), cls.end());
                add_projection(tb, ps, 0);
                if (hipMalloc(&dtab, std::max<size_t>(tb.buf.size(), 256)) != hipSuccess) {
                    rc = fail(KCS_EHIP, "tuning table");
                    break;
                }
                hipError_t e = hipMemcpy(dtab, tb.buf.data(), tb.buf.size(), hipMemcpyHostToDevice);
                float ms = 0.0f;
                for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // rep 0 warms up
                    if (rep == 1) e = hipEventRecord(e0, st);
                    for (const PlanPhase& ph : tb.phases)
                        if (e == hipSuccess) e = run_phase(ph, (const char*)dtab, st);
                }
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                (void)hipFree(dtab);
                dtab = nullptr;
                if (e != hipSuccess) {
                    rc = hip_fail(e, "projector tuning");
                    break;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = T;
                }
            }
            if (rc != KCS_OK) break;
            g_tuned.push_back({k, best});
            store_tile(k, best, best_ms / 3.0f);
        }
        for (StudyPrep* P : cls) P->T = best;
        if (rc == KCS_OK) rc = tune_lm_tile(cls, st, e0, e1);
        if (rc != KCS_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// ----- one ICM sweep, shared by the caller-workspace and the static-scratch entry points -----
int check_sweep_args(const kcs_geometry* g, const kcs_frames* f, const kcs_kinetics* k, const kcs_prior* p,
                     const kcs_lm_opts* lm, const float* d_sino, int32_t Q, int32_t sweep_idx, const float* d_x,
                     const float* d_params, const float* d_lambda) {
    KCS_TRY(check_geometry(g));
    KCS_TRY(check_frames(f));
    KCS_TRY(check_plane(g, f->n_frames));
    KCS_TRY(check_kinetics(k));
    KCS_TRY(check_prior(p, n_maps(*k)));
    KCS_TRY(check_lm(lm, n_maps(*k)));
    KCS_TRY(check_subset(g, 0, Q));
    if (sweep_idx < 0) return fail(KCS_EINVAL, "sweep_idx must be >= 0");
    if (!d_sino || !d_x || !d_params || !d_lambda) return fail(KCS_EINVAL, "device pointers must not be NULL");
    return KCS_OK;
}

// Every region of the workspace that the sweep reads is written earlier in the same sweep (the
// kinetic table, the model TACs, the ratio and partial sums of each subset, the ping-pong maps
// and the carried normal equations), so a workspace needs no clearing between calls.
int icm_sweep_body(const kcs_geometry& g, const kcs_frames& f, const kcs_kinetics& k, const kcs_prior& p,
                   const kcs_lm_opts& lm, const float* d_sino, int32_t Q, int32_t sweep_idx, float* d_x,
                   float* d_params, float* d_lambda, void* d_work, hipStream_t stream) {
    const Schedule S = make_schedule(f, &k);
    g_err.clear();
    KCS_TRY(do_setup(S, d_work, stream));
    const bool kp = p.kp_on != 0 && sweep_idx > 0;
    if (kp) KCS_TRY(do_model_pass(g, S, n_maps(k), d_params, d_work, Q, stream));
    for (int32_t q = 0; q < Q; ++q) KCS_TRY(do_osl(g, S, p, kp, d_sino, q, Q, d_x, d_work, stream));
    return do_lm(g, S, n_maps(k), p, lm, d_x, d_params, d_lambda, d_work, Q, lm.restart != 0, stream);
}

// ----- static scratch of kcs_icm_sweep_noalloc -----
// A workspace in the library's own device memory for callers that cannot allocate.  Each GPU
// holds its own copy from the load of the library to the end of the process.  In host code the
// array's name is not a device address: the address comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is passed to kernels.
constexpr size_t kScratchBytes = size_t(256) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(KCS_EINVAL, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0)
            return fail(KCS_EHIP, "static scratch has no 256-byte aligned device address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return KCS_OK;
}

}  // namespace
}  // namespace kcs

using namespace kcs;

struct kcs_plan {
    std::vector<PlanPhase> phases;
    std::vector<int> tiles;
    std::vector<int> lm_tiles;  // voxel tile width of the fit, per study
    int n_studies = 0;
    void* d_tables = nullptr;
    void* h_tables = nullptr;  // pinned staging of the tables (the upload is asynchronous)
    hipEvent_t ready = nullptr;  // recorded on the creation stream after setup and upload
    hipEvent_t done = nullptr;   // recorded after each run; destruction waits for it
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* kcs_last_error(void) { return g_err.c_str(); }

int kcs_timing_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    return KCS_OK;
}

int kcs_timing_collect(double* total_ms, int64_t* count) {
    if (!total_ms || !count) return fail(KCS_EINVAL, "output arrays must not be NULL");
    std::vector<TimedLaunch> ls;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        ls.swap(g_launches);
    }
    for (int k = 0; k < KCS_TIMING_KINDS; ++k) {
        total_ms[k] = 0.0;
        count[k] = 0;
    }
    int rc = KCS_OK;
    for (const TimedLaunch& t : ls) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess && rc == KCS_OK) rc = hip_fail(e, "timing event");
        total_ms[t.kind] += ms;
        count[t.kind] += 1;
    }
    std::lock_guard<std::mutex> lk(g_tmu);
    for (const TimedLaunch& t : ls) {
        g_event_pool.push_back(t.a);
        g_event_pool.push_back(t.b);
    }
    return rc;
}

int kcs_stream_probe(int32_t kind, const void* d_src, void* d_dst, size_t bytes, int32_t groups, hipStream_t stream) {
    if (kind != 0 && kind != 1) return fail(KCS_EINVAL, "kind must be 0 (read) or 1 (copy)");
    if (!d_src || !d_dst) return fail(KCS_EINVAL, "device pointers must not be NULL");
    if (bytes == 0 || bytes % 16 != 0) return fail(KCS_EINVAL, "bytes must be a positive multiple of 16");
    if ((reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst)) & 15)
        return fail(KCS_EINVAL, "pointers must be 16-byte aligned");
    if (groups < 1 || groups > (1 << 20)) return fail(KCS_EINVAL, "need 1 <= groups <= 2^20");
    if (kind == 1) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(d_src), b = reinterpret_cast<uintptr_t>(d_dst);
        if (a < b + bytes && b < a + bytes) return fail(KCS_EINVAL, "copy ranges overlap");
    }
    g_err.clear();
    return launched(launch_stream(kind, d_src, d_dst, bytes, groups, stream), "stream probe");
}

size_t kcs_workspace_bytes(const kcs_geometry* g, int32_t n_frames, int32_t Q) {
    if (g && check_geometry(g) != KCS_OK) return 0;
    if (Q < 0) Q = 0;
    return layout(g, n_frames > 0 ? n_frames : kMaxFrames, Q).total;
}

size_t kcs_study_footprint_bytes(const kcs_geometry* g, int32_t n_frames, int32_t Q) {
    if (!g || check_geometry(g) != KCS_OK) return 0;
    const size_t N = (size_t)g->nx * g->ny * g->nz;
    const size_t S = (size_t)g->nz * g->n_ang * g->n_bin * n_frames;
    const size_t mult = g->d_mult ? (size_t)g->nz * g->n_ang * g->n_bin : 0;
    return (S + N * n_frames + 3 * N + N + mult) * sizeof(float) + kcs_workspace_bytes(g, n_frames, Q);
}

int kcs_project(const kcs_geometry* g, const kcs_frames* f, const float* d_x, int32_t q, int32_t Q, float* d_ybar,
                hipStream_t stream) {
    KCS_TRY(check_geometry(g));
    KCS_TRY(check_frames(f));
    KCS_TRY(check_plane(g, f->n_frames));
    KCS_TRY(check_subset(g, q, Q));
    if (!d_x || !d_ybar) return fail(KCS_EINVAL, "device pointers must not be NULL");
    const Schedule S = make_schedule(*f, nullptr);
    g_err.clear();
    const ProjArgs pa = proj_args(*g, S.fr, q, Q);
    return launched(
        timed(KCS_T_PROJECT, stream, [&] { return launch_project(f->n_frames, d_x, nullptr, d_ybar, pa, false, stream); }),
        "forward projection");
}

int kcs_backproject(const kcs_geometry* g, const kcs_frames* f, const float* d_y, int32_t q, int32_t Q, float* d_b,
                    float* d_sens, hipStream_t stream) {
    KCS_TRY(check_geometry(g));
    KCS_TRY(check_frames(f));
    KCS_TRY(check_plane(g, f->n_frames));
    KCS_TRY(check_subset(g, q, Q));
    if (!d_y || !d_b) return fail(KCS_EINVAL, "device pointers must not be NULL");
    const Schedule S = make_schedule(*f, nullptr);
    g_err.clear();
    const ProjArgs pa = proj_args(*g, S.fr, q, Q);
    return launched(
        timed(KCS_T_BACK, stream, [&] { return launch_backproject(f->n_frames, d_y, d_b, d_sens, pa, stream); }),
        "back projection");
}

int kcs_model_tac(const kcs_frames* f, const kcs_kinetics* k, const float* d_params, int64_t n, float* d_F, float* d_J,
                  void* d_work, size_t work_bytes, hipStream_t stream) {
    KCS_TRY(check_frames(f));
    KCS_TRY(check_kinetics(k));
    if (n < 0) return fail(KCS_EINVAL, "n must be >= 0");
    if (n > 0 && (!d_params || !d_F)) return fail(KCS_EINVAL, "device pointers must not be NULL");
    KCS_TRY(check_work(nullptr, f->n_frames, 0, d_work, work_bytes));
    if (n == 0) return KCS_OK;
    const Schedule S = make_schedule(*f, k);
    g_err.clear();
    KCS_TRY(do_setup(S, d_work, stream));
    const KinTab* K = at<KinTab>(d_work, layout(nullptr, 0, 0).kin);
    return launched(
        timed(KCS_T_MODEL, stream,
              [&] { return launch_model(f->n_frames, n_maps(*k), K, S.fr, d_params, n, d_F, d_J, stream); }),
        "model evaluation");
}

int kcs_ki_map(const float* d_params, int64_t n, float* d_ki, hipStream_t stream) {
    if (n < 0) return fail(KCS_EINVAL, "n must be >= 0");
    if (n > (int64_t)INT32_MAX * 256) return fail(KCS_EINVAL, "n is too large (at most 2^31 - 1 workgroups of 256)");
    if (n > 0 && (!d_params || !d_ki)) return fail(KCS_EINVAL, "device pointers must not be NULL");
    if (n == 0) return KCS_OK;
    g_err.clear();
    return launched(launch_ki(d_params, n, d_ki, stream), "K_i map");
}

int kcs_rebin_ssrb(int32_t n_rings, int32_t max_ring_diff, int32_t n_ang, int32_t n_bin, int32_t n_frames,
                   const float* d_y3d, float* d_y2d, float* d_count, hipStream_t stream) {
    if (n_rings < 1 || n_rings > 4096) return fail(KCS_EINVAL, "n_rings must be in [1, 4096]");
    if (max_ring_diff < 0 || max_ring_diff > n_rings - 1) return fail(KCS_EINVAL, "need 0 <= max_ring_diff <= n_rings - 1");
    if (n_ang < 1 || n_bin < 1 || n_frames < 1) return fail(KCS_EINVAL, "n_ang, n_bin and n_frames must be >= 1");
    if (!d_y3d || !d_y2d) return fail(KCS_EINVAL, "device pointers must not be NULL");
    const double out_values = (double)(2 * n_rings - 1) * n_ang * n_bin * n_frames;
    if (out_values / 256.0 >= 4294967295.0) return fail(KCS_ESHAPE, "output too large for one launch");
    g_err.clear();
    const RebinArgs a{n_rings, max_ring_diff, n_ang, n_bin, n_frames};
    return launched(launch_ssrb(a, d_y3d, d_y2d, d_count, stream), "single-slice rebinning");
}

int kcs_osl_update(const kcs_geometry* g, const kcs_frames* f, const kcs_kinetics* k, const kcs_prior* p,
                   const float* d_sino, const float* d_params, int32_t q, int32_t Q, float* d_x, void* d_work,
                   size_t work_bytes, hipStream_t stream) {
    KCS_TRY(check_geometry(g));
    KCS_TRY(check_frames(f));
    KCS_TRY(check_plane(g, f->n_frames));
    KCS_TRY(check_kinetics(k));
    KCS_TRY(check_prior(p, n_maps(*k)));
    KCS_TRY(check_subset(g, q, Q));
    if (!d_sino || !d_x || (p->kp_on && !d_params)) return fail(KCS_EINVAL, "device pointers must not be NULL");
    KCS_TRY(check_work(g, f->n_frames, Q, d_work, work_bytes));
    const Schedule S = make_schedule(*f, k);
    g_err.clear();
    if (p->kp_on) {
        KCS_TRY(do_setup(S, d_work, stream));
        KCS_TRY(do_model_pass(*g, S, n_maps(*k), d_params, d_work, Q, stream));
    }
    return do_osl(*g, S, *p, p->kp_on != 0, d_sino, q, Q, d_x, d_work, stream);
}

int kcs_lm_fit(const kcs_geometry* g, const kcs_frames* f, const kcs_kinetics* k, const kcs_prior* p,
               const kcs_lm_opts* lm, const float* d_x, float* d_params, float* d_lambda, void* d_work,
               size_t work_bytes, hipStream_t stream) {
    KCS_TRY(check_geometry(g));
    KCS_TRY(check_frames(f));
    KCS_TRY(check_plane(g, f->n_frames));
    KCS_TRY(check_kinetics(k));
    KCS_TRY(check_prior(p, n_maps(*k)));
    KCS_TRY(check_lm(lm, n_maps(*k)));
    if (!d_x || !d_params || !d_lambda) return fail(KCS_EINVAL, "device pointers must not be NULL");
    KCS_TRY(check_work(g, f->n_frames, 0, d_work, work_bytes));
    const Schedule S = make_schedule(*f, k);
    g_err.clear();
    KCS_TRY(do_setup(S, d_work, stream));
    return do_lm(*g, S, n_maps(*k), *p, *lm, d_x, d_params, d_lambda, d_work, 0, false, stream);
}

int kcs_init_state(const kcs_geometry* g, const kcs_frames* f, const float* d_sino, const double* xi0, int32_t n_maps,
                   float* d_x, float* d_params, float* d_lambda, void* d_work, size_t work_bytes, hipStream_t stream) {
    KCS_TRY(check_geometry(g));
    KCS_TRY(check_frames(f));
    KCS_TRY(check_plane(g, f->n_frames));
    if (!d_sino || !d_x || !d_params || !d_lambda || !xi0) return fail(KCS_EINVAL, "pointers must not be NULL");
    if (n_maps != 3 && n_maps != 4) return fail(KCS_EINVAL, "n_maps must be 3 or 4");
    for (int i = 0; i < n_maps; ++i)
        if (!is_finite(xi0[i])) return fail(KCS_EINVAL, "xi0 must be finite");
    KCS_TRY(check_work(g, f->n_frames, 0, d_work, work_bytes));
    const Schedule S = make_schedule(*f, nullptr);
    const double sumP = total_path_length(*g);
    if (!(sumP > 0)) return fail(KCS_EINVAL, "no ray crosses the image");
    const Layout L = layout(g, f->n_frames, 0);
    const int64_t rows = (int64_t)g->nz * g->n_ang * g->n_bin;
    const int32_t N = g->nx * g->ny * g->nz;
    g_err.clear();
    return launched(timed(KCS_T_INIT, stream,
                          [&] {
                              return launch_init(f->n_frames, d_sino, rows, S.fr, sumP * g->nz, N, xi0, n_maps,
                                                 at<double>(d_work, L.init), kInitChunks, d_x, d_params, d_lambda,
                                                 stream);
                          }),
                    "initial state");
}

int kcs_icm_sweep(const kcs_geometry* g, const kcs_frames* f, const kcs_kinetics* k, const kcs_prior* p,
                  const kcs_lm_opts* lm, const float* d_sino, int32_t Q, int32_t sweep_idx, float* d_x, float* d_params,
                  float* d_lambda, void* d_work, size_t work_bytes, hipStream_t stream) {
    KCS_TRY(check_sweep_args(g, f, k, p, lm, d_sino, Q, sweep_idx, d_x, d_params, d_lambda));
    KCS_TRY(check_work(g, f->n_frames, Q, d_work, work_bytes));
    return icm_sweep_body(*g, *f, *k, *p, *lm, d_sino, Q, sweep_idx, d_x, d_params, d_lambda, d_work, stream);
}

int kcs_icm_sweep_noalloc(const kcs_geometry* g, const kcs_frames* f, const kcs_kinetics* k, const kcs_prior* p,
                          const kcs_lm_opts* lm, const float* d_sino, int32_t Q, int32_t sweep_idx, float* d_x,
                          float* d_params, float* d_lambda, hipStream_t stream) {
    KCS_TRY(check_sweep_args(g, f, k, p, lm, d_sino, Q, sweep_idx, d_x, d_params, d_lambda));
    const size_t need = layout(g, f->n_frames, Q).total;
    if (need > kScratchBytes)
        return fail(KCS_EWORKSPACE, "study needs %zu bytes of workspace; the library's static scratch holds %zu", need,
                    kScratchBytes);
    void* work = nullptr;
    KCS_TRY(scratch_address(&work));
    return icm_sweep_body(*g, *f, *k, *p, *lm, d_sino, Q, sweep_idx, d_x, d_params, d_lambda, work, stream);
}

int kcs_plan_create(const kcs_study* studies, int32_t n, int32_t flags, hipStream_t stream, kcs_plan** out) {
    if (!out) return fail(KCS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !studies) return fail(KCS_EINVAL, "need at least one study");
    std::vector<StudyPrep> preps(n);
    for (int i = 0; i < n; ++i) {
        const int rc = check_study(studies[i]);
        if (rc != KCS_OK) return fail(rc, "study %d: %s", i, g_err.c_str());
        preps[i].s = &studies[i];
        preps[i].S = make_schedule(studies[i].f, &studies[i].k);
        preps[i].L = layout(&studies[i].g, studies[i].f.n_frames, studies[i].Q);
        preps[i].T = projector_tile(studies[i].g, studies[i].f.n_frames, studies[i].Q);
    }
    g_err.clear();
    for (const StudyPrep& P : preps) KCS_TRY(do_setup(P.S, P.s->d_work, stream));
    if (flags & KCS_PLAN_AUTOTUNE) KCS_TRY(autotune(preps, stream));
    TableBuilder tb;
    build_schedule(tb, preps);
    kcs_plan* plan = new kcs_plan();
    plan->phases = tb.phases;
    for (const StudyPrep& P : preps) plan->tiles.push_back(P.T);
    for (const StudyPrep& P : preps) plan->lm_tiles.push_back(lm_tile_for(P.s->g.nx, P.s->g.ny));
    plan->n_studies = n;
    const size_t tbytes = std::max<size_t>(tb.buf.size(), 256);
    hipError_t e = hipMalloc(&plan->d_tables, tbytes);
    if (e == hipSuccess) e = hipHostMalloc(&plan->h_tables, tbytes, hipHostMallocDefault);
    if (e == hipSuccess) {
        memcpy(plan->h_tables, tb.buf.data(), tb.buf.size());
        e = hipMemcpyAsync(plan->d_tables, plan->h_tables, tb.buf.size(), hipMemcpyHostToDevice, stream);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(plan->ready, stream);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->done, hipEventDisableTiming);
    if (e == hipSuccess && (flags & KCS_PLAN_GRAPH)) {
        e = hipStreamCreateWithFlags(&plan->capture, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(plan->capture, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = hipSuccess;
            for (const PlanPhase& ph : plan->phases)
                if (le == hipSuccess) le = run_phase(ph, (const char*)plan->d_tables, plan->capture);
            e = hipStreamEndCapture(plan->capture, &plan->graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
        kcs_plan_destroy(plan);
        return hip_fail(e, "plan creation");
    }
    *out = plan;
    return KCS_OK;
}

int kcs_plan_run(kcs_plan* plan, hipStream_t stream) {
    if (!plan) return fail(KCS_EINVAL, "plan is NULL");
    g_err.clear();
    // order the run after the plan's setup and table upload when it goes on another stream
    if (hipEventQuery(plan->ready) != hipSuccess)
        KCS_TRY(launched(hipStreamWaitEvent(stream, plan->ready, 0), "wait for plan setup"));
    if (plan->exec) {
        KCS_TRY(launched(hipGraphLaunch(plan->exec, stream), "graph launch"));
    } else {
        for (const PlanPhase& ph : plan->phases)
            KCS_TRY(launched(run_phase(ph, (const char*)plan->d_tables, stream), "plan phase"));
    }
    return launched(hipEventRecord(plan->done, stream), "plan completion event");
}

int kcs_plan_describe(const kcs_plan* plan, char* buf, size_t len) {
    if (!plan || !buf || len == 0) return fail(KCS_EINVAL, "bad arguments");
    std::string t = "studies=" + std::to_string(plan->n_studies) + " launches=" + std::to_string(plan->phases.size()) +
                    " graph=" + (plan->exec ? "yes" : "no") + " tiles=";
    for (size_t i = 0; i < plan->tiles.size(); ++i) t += (i ? "," : "") + std::to_string(plan->tiles[i]);
    t += " lm_tiles=";
    for (size_t i = 0; i < plan->lm_tiles.size(); ++i) t += (i ? "," : "") + std::to_string(plan->lm_tiles[i]);
    snprintf(buf, len, "%s", t.c_str());
    return KCS_OK;
}

void kcs_plan_destroy(kcs_plan* plan) {
    if (!plan) return;
    // the tables may still be read by a run in flight, and the upload may still be pending
    if (plan->done) (void)hipEventSynchronize(plan->done);
    if (plan->ready) (void)hipEventSynchronize(plan->ready);
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->capture) (void)hipStreamDestroy(plan->capture);
    if (plan->d_tables) (void)hipFree(plan->d_tables);
    if (plan->h_tables) (void)hipHostFree(plan->h_tables);
    if (plan->ready) (void)hipEventDestroy(plan->ready);
    if (plan->done) (void)hipEventDestroy(plan->done);
    delete plan;
}

}  // extern "C"
