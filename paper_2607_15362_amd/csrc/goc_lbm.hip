// goc_lbm.hip -- host runtime and C-ABI of libgoclbm.so (see include/goc_lbm.h).
//
// The runtime owns, per handle: a table of run descriptors (one per
// independent run; the single-run API is a batch of one), pooled device
// state (two slot buffers for ping-pong, which hold the D2Q5 slots of MHD
// runs in their rows, and two lagged-force buffers),
// the metric pools (FP64), and HIP graphs of blocks of steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/goc_lbm.h"
#include "goc_aux.hpp"
#include "goc_tile.hpp"

using goc::RunDesc;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPOK(expr)                                                                          \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(GOC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

constexpr int kGraphSteps = 100;    // steps per captured graph

size_t storage_bytes(int storage)
{
    switch (storage) {
    case GOC_F64: return 8;
    case GOC_F32: return 4;
    default: return 2;
    }
}
size_t force_bytes(int storage) { return storage == GOC_F64 ? 8 : 4; }

// ---------------------------------------------------------------- metric --
// Host generation of h and dh/dxi at node centres xi = j + 1/2 (FP64) and
// of h on the two faces, for the analytic stretchings of Sec. 6.
struct Metric1D {
    std::vector<double> h, dh;
    double face_lo = 1.0, face_hi = 1.0;
};

int metric_1d(int n, int kind, double param, const double* harr, const double* dharr,
              const double* faces, bool periodic, Metric1D& out)
{
    out.h.assign(n, 1.0);
    out.dh.assign(n, 0.0);
    const double L = n;
    if (kind == GOC_STRETCH_UNIFORM || (kind == GOC_STRETCH_TANH && param == 0.0)) {
        out.face_lo = out.face_hi = 1.0;
        return GOC_OK;
    }
    if (kind == GOC_STRETCH_TANH) {
        // y = (L/2) {1 - tanh[beta (1 - 2 xi/L)] / tanh beta}
        const double b = param, c = b / std::tanh(b);
        if (!(b > 0)) return fail(GOC_EINVAL, "tanh stretching needs beta > 0 (got %g)", b);
        for (int j = 0; j < n; ++j) {
            const double u = b * (1.0 - 2.0 * (j + 0.5) / L);
            const double ch = std::cosh(u), s2 = 1.0 / (ch * ch);
            out.h[j] = c * s2;
            out.dh[j] = c * s2 * std::tanh(u) * (4.0 * b / L);
        }
        const double cb = std::cosh(b);
        out.face_lo = out.face_hi = c / (cb * cb);
        return GOC_OK;
    }
    if (kind == GOC_STRETCH_ROBERTS) {
        // y = L [A l - B] / [C (1 + l)], l = lambda^s, s = (xi/L - 1/2)/(1/2),
        // lambda = (gamma + 1)/(gamma - 1), A = gamma + 1, B = gamma - 1, C = 2
        const double g = param;
        if (!(g > 1.0)) return fail(GOC_EINVAL, "Roberts stretching needs gamma > 1 (got %g)", g);
        const double lam = (g + 1.0) / (g - 1.0), A = g + 1.0, B = g - 1.0, C = 2.0;
        const double k = std::log(lam) / (L * 0.5);
        auto hd = [&](double xi, double& h, double& dh) {
            const double s = (xi / L - 0.5) / 0.5, l = std::pow(lam, s);
            h = (L / C) * (A + B) * k * l / ((1 + l) * (1 + l));
            dh = (L / C) * (A + B) * k * k * l * (1 - l) / ((1 + l) * (1 + l) * (1 + l));
        };
        for (int j = 0; j < n; ++j) hd(j + 0.5, out.h[j], out.dh[j]);
        double t;
        hd(0.0, out.face_lo, t);
        hd(L, out.face_hi, t);
        return GOC_OK;
    }
    if (kind != GOC_STRETCH_ARRAY) return fail(GOC_EINVAL, "unknown stretch kind %d", kind);
    if (!harr) return fail(GOC_EINVAL, "array metric without h");
    for (int j = 0; j < n; ++j) {
        if (!(harr[j] > 0.0) || !std::isfinite(harr[j]))
            return fail(GOC_EINVAL, "metric factor h[%d] = %g must be positive", j, harr[j]);
        out.h[j] = harr[j];
    }
    if (dharr) {
        for (int j = 0; j < n; ++j) out.dh[j] = dharr[j];
    } else {
        // second-order differences: central, wrapped when periodic, one-sided at the ends
        for (int j = 0; j < n; ++j) {
            if (periodic) out.dh[j] = 0.5 * (out.h[(j + 1) % n] - out.h[(j + n - 1) % n]);
            else if (j == 0) out.dh[j] = 0.5 * (-3 * out.h[0] + 4 * out.h[1] - out.h[2]);
            else if (j == n - 1) out.dh[j] = 0.5 * (3 * out.h[n - 1] - 4 * out.h[n - 2] + out.h[n - 3]);
            else out.dh[j] = 0.5 * (out.h[j + 1] - out.h[j - 1]);
        }
    }
    out.face_lo = (faces && faces[0] > 0) ? faces[0] : out.h[0];
    out.face_hi = (faces && faces[1] > 0) ? faces[1] : out.h[n - 1];
    return GOC_OK;
}

bool is_2d(const goc_metric& m) { return m.kind_x == GOC_STRETCH_ANNULUS || m.kind_x == GOC_STRETCH_ARRAY2D; }

// A 2-D metric leaves the separable tables uniform (unused by its kernels).
int build_metric(const goc_grid& g, const goc_metric& m, Metric1D& mx, Metric1D& my)
{
    if (is_2d(m)) {
        int rc = metric_1d(g.nx, GOC_STRETCH_UNIFORM, 0.0, nullptr, nullptr, nullptr, false, mx);
        return rc ? rc : metric_1d(g.ny, GOC_STRETCH_UNIFORM, 0.0, nullptr, nullptr, nullptr, false, my);
    }
    int rc = metric_1d(g.nx, m.kind_x, m.param_x, m.h1, m.dh1, m.h1_face, g.bc_x == GOC_BC_PERIODIC, mx);
    if (rc) return rc;
    return metric_1d(g.ny, m.kind_y, m.param_y, m.h2, m.dh2, m.h2_face, g.bc_y == GOC_BC_PERIODIC, my);
}

// General 2-D metric at the nodes (FP64, row-major [ny][nx]): h1, h2 and
// their derivatives, with the face values h1 on the xi1 = 0 / nx faces per
// row and h2 on the xi2 = 0 / ny faces per column.
struct Metric2D {
    std::vector<double> h1, h2, d1h1, d2h1, d1h2, d2h2;
    std::vector<double> h1_lo, h1_hi, h2_lo, h2_hi;
    double qmin = 1.0;
};

int build_metric2d(const goc_grid& g, const goc_metric& m, Metric2D& out)
{
    const int nx = g.nx, ny = g.ny;
    const size_t N = (size_t)nx * ny;
    for (auto* v : {&out.h1, &out.h2, &out.d1h1, &out.d2h1, &out.d1h2, &out.d2h2}) v->assign(N, 0.0);
    out.h1_lo.assign(ny, 0.0);
    out.h1_hi.assign(ny, 0.0);
    out.h2_lo.assign(nx, 0.0);
    out.h2_hi.assign(nx, 0.0);
    if (m.kind_x == GOC_STRETCH_ANNULUS) {
        // Z = a exp(pi W / N_theta) on xi1 in [0, nx] (radii a .. Ro) and
        // xi2 in [0, ny] (angle 2 pi / N_theta): r = a exp(k xi1), k =
        // ln(Ro / a) / nx; h1 = dr/dxi1 = k r; h2 = r (2 pi / N_theta) / ny
        const double a = m.param_x, Ro = m.param_y, nt = m.n_theta;
        if (!(a > 0) || !(Ro > a) || !(nt > 0))
            return fail(GOC_EINVAL, "annulus needs 0 < a < Ro and n_theta > 0 (got %g, %g, %g)", a, Ro, nt);
        const double k = std::log(Ro / a) / nx, c2 = 2.0 * M_PI / (nt * ny);
        for (int i = 0; i < nx; ++i) {
            const double r = a * std::exp(k * (i + 0.5));
            for (int j = 0; j < ny; ++j) {
                const size_t n = (size_t)j * nx + i;
                out.h1[n] = k * r;
                out.h2[n] = c2 * r;
                out.d1h1[n] = k * k * r;
                out.d1h2[n] = k * c2 * r;
            }
            out.h2_lo[i] = out.h2_hi[i] = c2 * r;
        }
        for (int j = 0; j < ny; ++j) {
            out.h1_lo[j] = k * a;
            out.h1_hi[j] = k * Ro;
        }
    } else {
        if (!m.h1_2d || !m.h2_2d) return fail(GOC_EINVAL, "2-D array metric needs h1_2d and h2_2d");
        const int given = !!m.d1h1 + !!m.d2h1 + !!m.d1h2 + !!m.d2h2;
        if (given != 0 && given != 4) return fail(GOC_EINVAL, "give all four metric derivative arrays or none");
        for (size_t n = 0; n < N; ++n) {
            if (!(m.h1_2d[n] > 0) || !(m.h2_2d[n] > 0) || !std::isfinite(m.h1_2d[n]) || !std::isfinite(m.h2_2d[n]))
                return fail(GOC_EINVAL, "metric factors at node %zu must be positive", n);
            out.h1[n] = m.h1_2d[n];
            out.h2[n] = m.h2_2d[n];
        }
        if (given == 4) {
            for (size_t n = 0; n < N; ++n) {
                out.d1h1[n] = m.d1h1[n];
                out.d2h1[n] = m.d2h1[n];
                out.d1h2[n] = m.d1h2[n];
                out.d2h2[n] = m.d2h2[n];
            }
        } else {
            // second-order differences: central, wrapped along a periodic
            // axis, one-sided at the ends of a walled one
            auto dif = [&](const std::vector<double>& f, int i, int j, bool along_x) {
                const int n = along_x ? nx : ny, k = along_x ? i : j;
                auto v = [&](int t) { return along_x ? f[(size_t)j * nx + t] : f[(size_t)t * nx + i]; };
                const bool per = along_x ? g.bc_x == GOC_BC_PERIODIC : g.bc_y == GOC_BC_PERIODIC;
                if (per) return 0.5 * (v((k + 1) % n) - v((k + n - 1) % n));
                if (k == 0) return 0.5 * (-3 * v(0) + 4 * v(1) - v(2));
                if (k == n - 1) return 0.5 * (3 * v(n - 1) - 4 * v(n - 2) + v(n - 3));
                return 0.5 * (v(k + 1) - v(k - 1));
            };
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const size_t n = (size_t)j * nx + i;
                    out.d1h1[n] = dif(out.h1, i, j, true);
                    out.d2h1[n] = dif(out.h1, i, j, false);
                    out.d1h2[n] = dif(out.h2, i, j, true);
                    out.d2h2[n] = dif(out.h2, i, j, false);
                }
        }
        for (int j = 0; j < ny; ++j) {
            out.h1_lo[j] = out.h1[(size_t)j * nx];
            out.h1_hi[j] = out.h1[(size_t)j * nx + nx - 1];
        }
        for (int i = 0; i < nx; ++i) {
            out.h2_lo[i] = out.h2[i];
            out.h2_hi[i] = out.h2[(size_t)(ny - 1) * nx + i];
        }
    }
    out.qmin = std::min(*std::min_element(out.h1.begin(), out.h1.end()),
                        *std::min_element(out.h2.begin(), out.h2.end()));
    return GOC_OK;
}

// Node planes of a 2-D run (goc::M_*), FP64, with P0 = rho0 c_s^2 for the
// rest-state offsets of the axis slots.
void metric2d_planes(const goc_grid& g, const Metric2D& m, double P0, double* out)
{
    const int nx = g.nx, ny = g.ny;
    const size_t N = (size_t)nx * ny;
    const bool px = g.bc_x == GOC_BC_PERIODIC, py = g.bc_y == GOC_BC_PERIODIC;
    auto r21 = [&](int i, int j) { const size_t n = (size_t)j * nx + i; return m.h2[n] / m.h1[n]; };
    auto r12 = [&](int i, int j) { const size_t n = (size_t)j * nx + i; return m.h1[n] / m.h2[n]; };
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t n = (size_t)j * nx + i;
            const double h1 = m.h1[n], h2 = m.h2[n];
            out[goc::M_H1 * N + n] = h1;
            out[goc::M_IH1 * N + n] = 1.0 / h1;
            out[goc::M_H2 * N + n] = h2;
            out[goc::M_IH2 * N + n] = 1.0 / h2;
            out[goc::M_TH11 * N + n] = m.d1h1[n] / (h1 * h1);
            out[goc::M_TH12 * N + n] = m.d2h1[n] / (h1 * h2);
            out[goc::M_TH21 * N + n] = m.d1h2[n] / (h1 * h2);
            out[goc::M_TH22 * N + n] = m.d2h2[n] / (h2 * h2);
            const int ie = i + 1 < nx ? i + 1 : (px ? 0 : -1);
            const int iw = i > 0 ? i - 1 : (px ? nx - 1 : -1);
            const int jn = j + 1 < ny ? j + 1 : (py ? 0 : -1);
            const int js = j > 0 ? j - 1 : (py ? ny - 1 : -1);
            out[goc::M_AE * N + n] = ie < 0 ? 0.0 : 0.5 * P0 * (r21(i, j) - r21(ie, j));
            out[goc::M_AW * N + n] = iw < 0 ? 0.0 : 0.5 * P0 * (r21(i, j) - r21(iw, j));
            out[goc::M_AN * N + n] = jn < 0 ? 0.0 : 0.5 * P0 * (r12(i, j) - r12(i, jn));
            out[goc::M_AS * N + n] = js < 0 ? 0.0 : 0.5 * P0 * (r12(i, j) - r12(i, js));
        }
}

int check_grid(const goc_grid* g)
{
    if (!g) return fail(GOC_EINVAL, "grid is NULL");
    if (g->nx < 3 || g->ny < 3) return fail(GOC_EINVAL, "grid %d x %d: both sizes must be >= 3", g->nx, g->ny);
    if ((g->bc_x != 0 && g->bc_x != 1) || (g->bc_y != 0 && g->bc_y != 1))
        return fail(GOC_EINVAL, "boundary kinds must be GOC_BC_PERIODIC or GOC_BC_WALL");
    if ((int64_t)g->nx * g->ny > (int64_t)1 << 31) return fail(GOC_EINVAL, "grid too large");
    return GOC_OK;
}

}  // namespace

// ------------------------------------------------------------------ handle --
struct goc_lbm {
    int storage = GOC_F32;
    hipStream_t stream = nullptr;
    int device = 0;
    int nruns = 0;
    bool any_mhd = false;
    int coll = goc::kCollCentral;   // collision body of the step kernel
    bool m2d = false;               // runs on general 2-D metrics (curvilinear step)
    std::vector<Metric2D> m2;
    double* met_d = nullptr;        // 2-D metric planes, FP64 and FP32
    float* metf_d = nullptr;
    double* face_d = nullptr;       // 2-D metric face values
    std::vector<RunDesc> runs;
    std::vector<goc_params> params;
    std::vector<goc_grid> grids;
    std::vector<Metric1D> mx, my;
    std::vector<double> q;
    RunDesc* runs_d = nullptr;
    int32_t* block_run_d = nullptr;
    int total_blocks = 0;
    double *h1_d = nullptr, *th11_d = nullptr, *h2_d = nullptr, *th22_d = nullptr;
    double *col_d = nullptr, *row_d = nullptr;   // per-column / per-row tables
    float *colf_d = nullptr, *rowf_d = nullptr;   // their FP32 copies
    void* f[2] = {nullptr, nullptr};
    void* F[2] = {nullptr, nullptr};
    size_t f_elems = 0, F_elems = 0;   // (an MHD run's D2Q5 planes lie in the rows of the slot pool)
    int cur = 0;
    int64_t step = 0;
    int64_t watchdog = 1000;        // check for non-finite values at step return (0: never)
    int64_t watch_last = 0;         // step of the last check
    double* diag_part = nullptr;
    double* diag_out = nullptr;
    int diag_cap = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int rows_per_seg = 0;
    uint32_t* step_ctr = nullptr;   // device: index of the next step's rounding draws
    int ncu = 256;                  // compute units of the device
    double waves_per_cu = 16.0;     // launch plan: work-groups per CU over the whole launch
    bool tiled = false;             // straight runs stepped by the tiled kernel instead of the march
    int32_t* tile_first_d = nullptr;   // device: first tile of each run of the tiled kernel, then the total
    int32_t total_tiles = 0;
    int tile_rows = 8;              // rows of a tile of the tiled step (goc::kTileRows)
    int tile_cols = goc::kTileX;    // its columns (goc::kTileX, or goc::kTileXWide at 4 rows)
    bool tile_nt = false;           // the tiled step stores non-temporally
    int block_cap = 0;              // capacity of block_run_d (entries)
    // 16-bit storage: reference tables (the one in use, and the next one
    // while it is built), rows of all runs x kRef floats, and the step of
    // the last initialisation, from which the refresh points count
    float* ref_d[2] = {nullptr, nullptr};
    int64_t ref_rows = 0;
    int64_t ref_base = 0;
};

namespace {

template <class S>
using PoolsOf = goc::Pools<S, typename goc::ForceOf<S>::type>;

template <class S>
PoolsOf<S> pools(const goc_lbm* h, int in)
{
    using FT = typename goc::ForceOf<S>::type;
    PoolsOf<S> p;
    p.fin = static_cast<const S*>(h->f[in]);
    p.fout = static_cast<S*>(h->f[1 - in]);
    p.Fin = static_cast<const FT*>(h->F[in]);
    p.Fout = static_cast<FT*>(h->F[1 - in]);
    p.gin = p.fin;   // (the D2Q5 planes lie in the rows of the slot pool)
    p.gout = p.fout;
    p.col = h->col_d;
    p.row = h->row_d;
    p.colf = h->colf_d;
    p.rowf = h->rowf_d;
    p.met = h->met_d;
    p.metf = h->metf_d;
    p.face = h->face_d;
    p.ref_in = h->ref_d[0];
    p.ref_out = h->ref_d[0];
    return p;
}

// 16-bit deviation storage (stored relative to the reference table).
bool scaled_storage(int storage) { return storage == GOC_F16DEV || storage == GOC_BF16DEV; }

template <class Fn>
int dispatch(int storage, Fn&& fn)
{
    switch (storage) {
    case GOC_F64: return fn(double{});
    case GOC_F32: return fn(float{});
    case GOC_F16DEV: return fn(__half{});
    case GOC_BF16DEV: return fn(__hip_bfloat16{});
    default: return fail(GOC_EINVAL, "unknown storage %d", storage);
    }
}

// Launch one time step of every run (input buffer h->cur); k is the step's
// offset from the device step counter.  refresh (16-bit storage): build the
// next reference table from the current state first, encode this step's
// output with it, and let it take over afterwards.
int launch_step(goc_lbm* h, int k, bool refresh = false)
{
    return dispatch(h->storage, [&](auto tag) -> int {
        using S = decltype(tag);
        auto pl = pools<S>(h, h->cur);
        if constexpr (goc::Store<S>::scaled) {
            if (refresh) {
                hipLaunchKernelGGL(goc::ref_kernel<S>, dim3((unsigned)h->ref_rows), dim3(256), 0, h->stream,
                                   h->runs_d, h->nruns, pl, h->ref_d[1]);
                HIPOK(hipGetLastError());
                pl.ref_out = h->ref_d[1];
            }
        }
        if (h->m2d || h->tiled) {   // tiled step: one launch for every run
            const bool raw = h->coll == goc::kCollRaw;
            auto tiled = [&](auto cols, auto rows, auto nts) {
                constexpr int TX = decltype(cols)::value;
                constexpr int TY = decltype(rows)::value;
                constexpr bool NT = decltype(nts)::value;
                const dim3 cg(h->total_tiles), cb(TX, TY);
                auto go = [&](auto kernel) {
                    hipLaunchKernelGGL(kernel, cg, cb, 0, h->stream, h->runs_d, h->tile_first_d, h->nruns, pl,
                                       h->step_ctr, k);
                };
                if constexpr (sizeof(S) == 8 && TY > 8) {   // (FP64: at most 8 rows, see tile_shape_built)
                    return;
                } else if (h->m2d) {
                    if constexpr (TX == goc::kTileX) {   // (2-D metrics: 64 columns only)
                        raw ? go(goc::tile_step_kernel<S, goc::kCollRaw, true, false, TY, NT>)
                            : go(goc::tile_step_kernel<S, goc::kCollCentral, true, false, TY, NT>);
                    }
                } else if (h->any_mhd) {
                    raw ? go(goc::tile_step_kernel<S, goc::kCollRaw, false, true, TY, NT, TX>)
                        : go(goc::tile_step_kernel<S, goc::kCollCentral, false, true, TY, NT, TX>);
                } else {
                    raw ? go(goc::tile_step_kernel<S, goc::kCollRaw, false, false, TY, NT, TX>)
                        : go(goc::tile_step_kernel<S, goc::kCollCentral, false, false, TY, NT, TX>);
                }
            };
            auto tiled_nt = [&](auto cols, auto rows) {
                if (h->tile_nt) tiled(cols, rows, std::true_type{});
                else tiled(cols, rows, std::false_type{});
            };
            const std::integral_constant<int, goc::kTileX> narrow{};
            if (h->tile_cols == goc::kTileXWide && h->tile_rows == goc::kTileRowsWide && !h->m2d) {
                tiled_nt(std::integral_constant<int, goc::kTileXWide>{},
                         std::integral_constant<int, goc::kTileRowsWide>{});
            } else if (h->tile_cols != goc::kTileX) {
                return fail(GOC_EINVAL, "tile shape %d x %d not built", h->tile_cols, h->tile_rows);
            } else {
                switch (h->tile_rows) {
                case 4: tiled_nt(narrow, std::integral_constant<int, 4>{}); break;
                case 8: tiled_nt(narrow, std::integral_constant<int, 8>{}); break;
                case 16: tiled_nt(narrow, std::integral_constant<int, 16>{}); break;
                default: return fail(GOC_EINVAL, "tile height %d not built", h->tile_rows);
                }
            }
            HIPOK(hipGetLastError());
            if (goc::Store<S>::scaled && refresh) {
                const int64_t n = h->ref_rows * goc::kRef;
                hipLaunchKernelGGL(goc::copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream,
                                   h->ref_d[1], h->ref_d[0], n);
                HIPOK(hipGetLastError());
            }
            return GOC_OK;
        }
        if constexpr (goc::Store<S>::scaled)   // (16-bit storage steps with the tiled kernel only)
            return fail(GOC_EINVAL, "16-bit storage steps with the tiled kernel only");
        const dim3 grid(h->total_blocks), block(goc::kWave);
        const bool raw = h->coll == goc::kCollRaw;
        if (h->any_mhd && raw)
            hipLaunchKernelGGL((goc::step_kernel<S, true, goc::kCollRaw>), grid, block, 0, h->stream,
                               h->runs_d, h->block_run_d, pl, h->step_ctr, k);
        else if (h->any_mhd)
            hipLaunchKernelGGL((goc::step_kernel<S, true, goc::kCollCentral>), grid, block, 0, h->stream,
                               h->runs_d, h->block_run_d, pl, h->step_ctr, k);
        else if (raw)
            hipLaunchKernelGGL((goc::step_kernel<S, false, goc::kCollRaw>), grid, block, 0, h->stream,
                               h->runs_d, h->block_run_d, pl, h->step_ctr, k);
        else
            hipLaunchKernelGGL((goc::step_kernel<S, false, goc::kCollCentral>), grid, block, 0, h->stream,
                               h->runs_d, h->block_run_d, pl, h->step_ctr, k);
        HIPOK(hipGetLastError());
        return GOC_OK;
    });
}

// Device step counter: set to v, or advanced by v.
int counter_op(goc_lbm* h, uint32_t v, int add)
{
    hipLaunchKernelGGL(goc::counter_kernel, dim3(1), dim3(64), 0, h->stream, h->step_ctr, v, add);
    HIPOK(hipGetLastError());
    return GOC_OK;
}

int per_node_grid(const RunDesc& d, dim3& grid, dim3& block)
{
    block = dim3(256);
    grid = dim3((d.nx + 255) / 256, d.ny);
    return GOC_OK;
}

int free_all(goc_lbm* h)
{
    for (int k = 0; k < 2; ++k) {
        if (h->graph[k]) (void)hipGraphExecDestroy(h->graph[k]);
        (void)hipFree(h->f[k]);
        (void)hipFree(h->F[k]);
        (void)hipFree(h->ref_d[k]);
    }
    (void)hipFree(h->runs_d);
    (void)hipFree(h->block_run_d);
    (void)hipFree(h->h1_d);
    (void)hipFree(h->th11_d);
    (void)hipFree(h->h2_d);
    (void)hipFree(h->th22_d);
    (void)hipFree(h->col_d);
    (void)hipFree(h->row_d);
    (void)hipFree(h->colf_d);
    (void)hipFree(h->rowf_d);
    (void)hipFree(h->diag_part);
    (void)hipFree(h->diag_out);
    (void)hipFree(h->step_ctr);
    (void)hipFree(h->met_d);
    (void)hipFree(h->metf_d);
    (void)hipFree(h->face_d);
    (void)hipFree(h->tile_first_d);
    return GOC_OK;
}

int check_params(const goc_params* p, const goc_grid* g, int run)
{
    if (!p) return fail(GOC_EINVAL, "params is NULL");
    if (p->collision < GOC_COLL_CENTRAL || p->collision > GOC_COLL_SRT)
        return fail(GOC_EINVAL, "run %d: unknown collision model %d", run, p->collision);
    for (int k = 0; k < 9; ++k) {
        if (p->collision == GOC_COLL_SRT && k != 4) continue;   // SRT: one rate
        if (!(p->omega[k] > 0.0 && p->omega[k] < 2.0))
            return fail(GOC_EINVAL, "run %d: omega[%d] = %g outside (0, 2)", run, k, p->omega[k]);
    }
    if (p->collision == GOC_COLL_SRT && p->rho_terms)
        return fail(GOC_EINVAL, "run %d: the SRT model takes rho_terms = 0", run);
    if (!(p->rho0 > 0.0)) return fail(GOC_EINVAL, "run %d: rho0 must be positive", run);
    if (p->mhd && !(p->tau_m > 0.5)) return fail(GOC_EINVAL, "run %d: tau_m must exceed 1/2", run);
    if (p->mhd && !(p->mu_m > 0.0)) return fail(GOC_EINVAL, "run %d: mu_m must be positive", run);
    if (!std::isfinite(p->F_ext[0]) || !std::isfinite(p->F_ext[1]) || !std::isfinite(p->B0))
        return fail(GOC_EINVAL, "run %d: non-finite forcing", run);
    (void)g;
    return GOC_OK;
}

int choose_rows(int ny, int strips, int target_waves)
{
    // rows per y-segment: enough work-groups to fill the chip, at least 4 rows
    int segs = std::max(1, target_waves / std::max(1, strips));
    int rows = std::max(4, (ny + segs - 1) / segs);
    return rows;
}

// Launch plan: each run gets work-groups (64-column strips x row segments)
// in proportion to its nodes, about waves_per_cu per CU over the launch;
// fills segs / first_block of the runs and the work-group -> run list.
void plan_rows(goc_lbm* h, std::vector<int32_t>& block_run)
{
    int64_t total_nodes = 0;
    for (const RunDesc& d : h->runs) total_nodes += (int64_t)d.nx * d.ny;
    block_run.clear();
    for (int r = 0; r < h->nruns; ++r) {
        RunDesc& d = h->runs[r];
        const double share = double((int64_t)d.nx * d.ny) / double(total_nodes);
        const int target = std::max(1, int(share * h->waves_per_cu * h->ncu));
        const int rows = choose_rows(d.ny, d.strips, target);
        d.segs = std::max(1, std::min(goc::row_groups(d.ny), (d.ny + rows - 1) / rows));
        d.first_block = (int)block_run.size();
        for (int b = 0; b < d.strips * d.segs; ++b) block_run.push_back(r);
    }
    h->total_blocks = (int)block_run.size();
}

// The tiled kernel can step every handle on straight metrics (and is the
// only form on 2-D metrics).
bool tile_eligible(const goc_lbm* h) { return !h->m2d; }
// First tile of every run of the tiled step (and the total) for the
// handle's tile shape.
void tile_table(const goc_lbm* h, std::vector<int32_t>& tile_first, bool& overflow)
{
    tile_first.assign(h->nruns + 1, 0);
    overflow = false;
    for (int r = 0; r < h->nruns; ++r) {
        const int64_t gx = (h->runs[r].nx + h->tile_cols - 1) / h->tile_cols;
        const int64_t nt = gx * ((h->runs[r].ny + h->tile_rows - 1) / h->tile_rows);
        if ((int64_t)tile_first[r] + nt > INT32_MAX) overflow = true;
        tile_first[r + 1] = overflow ? 0 : tile_first[r] + (int32_t)nt;
    }
}

// Tile shapes built for a storage: 64 columns x 4, 8 and 16 rows (FP64 up
// to 8: at 16 rows, 1024 threads per work-group, its registers would
// spill), and 128 x 4 on straight grids.
bool tile_shape_built(int cols, int rows, int storage, bool m2d)
{
    if (cols == goc::kTileXWide) return rows == goc::kTileRowsWide && !m2d;
    if (cols != goc::kTileX) return false;
    if (storage == GOC_F64 && rows > 8) return false;
    for (int r : goc::kTileRows)
        if (r == rows) return true;
    return false;
}

void drop_graphs(goc_lbm* h)
{
    for (int k = 0; k < 2; ++k)
        if (h->graph[k]) {
            (void)hipGraphExecDestroy(h->graph[k]);
            h->graph[k] = nullptr;
        }
}

// Step an eligible handle with the tiled kernel, with tiles of `cols` x
// `rows` nodes (0: the current shape) and non-temporal stores or not
// (nt < 0: as now); synchronous, captured step graphs are dropped.
int use_tiled(goc_lbm* h, int cols = 0, int rows = 0, int nt = -1)
{
    HIPOK(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    h->tiled = true;
    if (nt >= 0) h->tile_nt = nt != 0;
    if (!cols) cols = h->tile_cols;
    if (!rows) rows = h->tile_rows;
    if (cols != h->tile_cols || rows != h->tile_rows) {
        const int old_cols = h->tile_cols, old_rows = h->tile_rows;
        h->tile_cols = cols;
        h->tile_rows = rows;
        std::vector<int32_t> tf;
        bool overflow;
        tile_table(h, tf, overflow);
        if (overflow) {
            h->tile_cols = old_cols;
            h->tile_rows = old_rows;
            return fail(GOC_EINVAL, "too many tiles in the launch");
        }
        HIPOK(hipMemcpy(h->tile_first_d, tf.data(), (h->nruns + 1) * 4, hipMemcpyHostToDevice));
        h->total_tiles = tf[h->nruns];
    }
    return GOC_OK;
}

// Apply a launch plan of the march on the device: run table and work list
// (synchronous; captured step graphs are dropped, as their grid changes).
int apply_plan(goc_lbm* h, double waves_per_cu)
{
    h->tiled = false;
    h->waves_per_cu = waves_per_cu;
    std::vector<int32_t> block_run;
    plan_rows(h, block_run);
    if ((int)block_run.size() > h->block_cap) {
        (void)hipFree(h->block_run_d);
        h->block_run_d = nullptr;
        h->block_cap = 0;
        if (hipMalloc(&h->block_run_d, block_run.size() * 4) != hipSuccess)
            return fail(GOC_ENOMEM, "hipMalloc of the work list failed");
        h->block_cap = (int)block_run.size();
    }
    HIPOK(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    HIPOK(hipMemcpy(h->runs_d, h->runs.data(), h->nruns * sizeof(RunDesc), hipMemcpyHostToDevice));
    HIPOK(hipMemcpy(h->block_run_d, block_run.data(), block_run.size() * 4, hipMemcpyHostToDevice));
    return GOC_OK;
}

int create_impl(goc_lbm_t** out, int nruns, const goc_grid* grid, const goc_metric* metric,
                const goc_params* params, int32_t storage, void* stream)
{
    if (!out) return fail(GOC_EINVAL, "out is NULL");
    *out = nullptr;
    if (nruns < 1) return fail(GOC_EINVAL, "nruns must be >= 1");
    if (storage < GOC_F64 || storage > GOC_BF16DEV) return fail(GOC_EINVAL, "unknown storage %d", storage);
    if (!grid || !metric || !params) return fail(GOC_EINVAL, "NULL grid, metric or params");
    auto* h = new (std::nothrow) goc_lbm();
    if (!h) return fail(GOC_ENOMEM, "host allocation failed");
    h->storage = storage;
    h->stream = static_cast<hipStream_t>(stream);
    h->nruns = nruns;
    int rc = GOC_OK;
    auto bail = [&](int code) {
        free_all(h);
        delete h;
        return code;
    };
    // validate every run before touching the device
    for (int r = 0; r < nruns; ++r) {
        Metric1D tx, ty;
        if ((rc = check_grid(&grid[r])) != GOC_OK) return bail(rc);
        if ((rc = check_params(&params[r], &grid[r], r)) != GOC_OK) return bail(rc);
        if ((rc = build_metric(grid[r], metric[r], tx, ty)) != GOC_OK) return bail(rc);
        if (params[r].collision != params[0].collision)
            return bail(fail(GOC_EINVAL, "run %d: the runs of a batch share one collision model", r));
        if (is_2d(metric[r]) != is_2d(metric[0]))
            return bail(fail(GOC_EINVAL, "run %d: the runs of a batch share the metric kind (2-D or straight)", r));
        if (is_2d(metric[r]) && params[r].mhd)
            return bail(fail(GOC_EINVAL, "run %d: MHD runs need a straight metric", r));
        // the step kernel addresses a run's slot region (Q planes of padded
        // rows, two ghost rows; Q = 20 with the D2Q5 slots in its rows) with
        // 32-bit byte offsets
        const int64_t row = goc::padded_row(grid[r].nx);
        const int64_t region = (params[r].mhd ? 2 * goc::kGPlanes : 9) * row * (grid[r].ny + 2) + 256;
        if (region * (int64_t)storage_bytes(storage) > (int64_t)UINT32_MAX)
            return bail(fail(GOC_EINVAL, "run %d: grid %d x %d too large for this storage "
                             "(slot region of one run above 4 GiB)", r, grid[r].nx, grid[r].ny));
    }
    h->m2d = is_2d(metric[0]);
    if (h->m2d) {
        h->m2.resize(nruns);
        for (int r = 0; r < nruns; ++r)
            if ((rc = build_metric2d(grid[r], metric[r], h->m2[r])) != GOC_OK) return bail(rc);
    }
    h->coll = params[0].collision == GOC_COLL_CENTRAL ? goc::kCollCentral : goc::kCollRaw;
    if (hipGetDevice(&h->device) != hipSuccess) return bail(fail(GOC_EDEVICE, "no HIP device"));
    int ncu = 256;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    const size_t sb = storage_bytes(storage), fb = force_bytes(storage);
    h->runs.resize(nruns);
    h->params.assign(params, params + nruns);
    h->grids.assign(grid, grid + nruns);
    h->mx.resize(nruns);
    h->my.resize(nruns);
    h->q.resize(nruns);
    int64_t sum_nx = 0, sum_ny = 0, f_elems = 0, F_elems = 0;
    int64_t met_elems = 0, face_elems = 0;
    // one wave per work-group; aim for ~16 waves per CU over the whole batch
    std::vector<int32_t> block_run;
    for (int r = 0; r < nruns; ++r) {
        if ((rc = check_grid(&grid[r])) != GOC_OK) return bail(rc);
        if ((rc = check_params(&params[r], &grid[r], r)) != GOC_OK) return bail(rc);
        if ((rc = build_metric(grid[r], metric[r], h->mx[r], h->my[r])) != GOC_OK) return bail(rc);
        const goc_grid& g = grid[r];
        const goc_params& p = params[r];
        RunDesc& d = h->runs[r];
        std::memset(&d, 0, sizeof(d));
        d.nx = g.nx;
        d.ny = g.ny;
        const int32_t row = int32_t(goc::padded_row(g.nx));
        d.bc_x = g.bc_x;
        d.bc_y = g.bc_y;
        // rows interleaved: the planes of a row lie together (row stride
        // Q * plane).  A plain run's row holds its 9 population planes; an
        // MHD run's row holds them, one unused plane and the 10 D2Q5 planes
        // (Q = 20): the step then streams one region per buffer rather than
        // two, which HBM serves faster (the step's memory pattern without
        // arithmetic, 4096 x 1024 FP32 with 128 x 4 tiles: 131.5 us per launch
        // with the D2Q5 slots in a pool of their own, 127.5 us interleaved)
        d.plane = row;
        d.pitch = (p.mhd ? 2 * goc::kGPlanes : 9) * row;
        d.pitchF = 2 * row;
        // slot regions (populations and D2Q5 slots) hold two ghost rows, -1 and ny, for
        // the step kernel's pulls beyond the domain in y
        const int64_t region = (int64_t)d.pitch * (g.ny + 2) + 256, regionF = (int64_t)d.pitchF * g.ny + 256;
        // the step kernel addresses a run's regions with 32-bit byte offsets
        if (region * (int64_t)sb > (int64_t)UINT32_MAX)
            return bail(fail(GOC_EINVAL, "run %d: grid %d x %d too large for this storage "
                             "(slot region of one run above 4 GiB)", r, g.nx, g.ny));
        d.f_off = f_elems + d.pitch;   // row 0 (row -1 before it)
        d.F_off = F_elems;
        d.g_off = d.f_off + (p.mhd ? goc::kGPlanes * row : 0);   // (the D2Q5 planes share the slot pool)
        f_elems += region;
        F_elems += regionF;
        if (p.mhd) h->any_mhd = true;
        d.col_off = sum_nx;
        d.row_off = sum_ny;
        d.metric2d = h->m2d ? 1 : 0;
        d.met_off = met_elems;
        d.face_off = face_elems;
        if (h->m2d) {
            met_elems += (int64_t)goc::kMet * g.nx * g.ny;
            face_elems += 2 * (int64_t)(g.nx + g.ny);
        }
        sum_nx += g.nx;
        sum_ny += g.ny;
        d.gi_terms = p.gi_terms;
        d.q3_sign = p.q3_sign;
        d.rho_terms = p.rho_terms;
        d.lid_corners = p.lid_corners;
        d.mhd = p.mhd;
        // SRT: every moment relaxes at omega[4] = 1/tau (so zeta = nu)
        for (int k = 0; k < 9; ++k) d.omega[k] = p.collision == GOC_COLL_SRT ? p.omega[4] : p.omega[k];
        d.Fx1 = p.F_ext[0];
        d.Fx2 = p.F_ext[1];
        d.rho0 = p.rho0;
        d.uw_lo = g.bc_y ? g.u_wall_lo : 0.0;
        d.uw_hi = g.bc_y ? g.u_wall_hi : 0.0;
        d.vw_lo = g.bc_x ? g.v_wall_lo : 0.0;
        d.vw_hi = g.bc_x ? g.v_wall_hi : 0.0;
        if (!std::isfinite(d.uw_lo) || !std::isfinite(d.uw_hi) || !std::isfinite(d.vw_lo) || !std::isfinite(d.vw_hi))
            return bail(fail(GOC_EINVAL, "run %d: non-finite wall speed", r));
        d.hw_lo = h->my[r].face_lo;
        d.hw_hi = h->my[r].face_hi;
        d.h1w_lo = h->mx[r].face_lo;
        d.h1w_hi = h->mx[r].face_hi;
        d.tau_m = p.mhd ? p.tau_m : 1.0;
        d.inv_mu = p.mhd ? 1.0 / p.mu_m : 1.0;
        d.B0 = p.mhd ? p.B0 : 0.0;
        d.strips = (g.nx + goc::kOwn - 1) / goc::kOwn;
    }
    h->ncu = ncu;
    plan_rows(h, block_run);
    h->block_cap = (int)block_run.size();
    // the tiled step: the faster form for a single straight run, and the
    // only form of the 16-bit storage (whose reference table it applies)
    h->tiled = tile_eligible(h) && (nruns == 1 || scaled_storage(storage));
    h->f_elems = f_elems;
    h->F_elems = F_elems;

    // metric pools and the FP64 precompute (theta, q)
    std::vector<double> h1(sum_nx), dh1(sum_nx), h2(sum_ny), dh2(sum_ny);
    for (int r = 0; r < nruns; ++r) {
        std::copy(h->mx[r].h.begin(), h->mx[r].h.end(), h1.begin() + h->runs[r].col_off);
        std::copy(h->mx[r].dh.begin(), h->mx[r].dh.end(), dh1.begin() + h->runs[r].col_off);
        std::copy(h->my[r].h.begin(), h->my[r].h.end(), h2.begin() + h->runs[r].row_off);
        std::copy(h->my[r].dh.begin(), h->my[r].dh.end(), dh2.begin() + h->runs[r].row_off);
    }
    double *dh1_d = nullptr, *dh2_d = nullptr, *bmin_d = nullptr;
    auto dev_alloc = [&](void** p, size_t bytes) -> int {
        if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess)
            return fail(GOC_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
        return GOC_OK;
    };
    if ((rc = dev_alloc((void**)&h->h1_d, sum_nx * 8)) || (rc = dev_alloc((void**)&h->th11_d, sum_nx * 8)) ||
        (rc = dev_alloc((void**)&h->h2_d, sum_ny * 8)) || (rc = dev_alloc((void**)&h->th22_d, sum_ny * 8)) ||
        (rc = dev_alloc((void**)&dh1_d, sum_nx * 8)) || (rc = dev_alloc((void**)&dh2_d, sum_ny * 8)) ||
        (rc = dev_alloc((void**)&h->col_d, sum_nx * goc::kTab * 8)) ||
        (rc = dev_alloc((void**)&h->row_d, sum_ny * goc::kTab * 8)) ||
        (rc = dev_alloc((void**)&h->colf_d, sum_nx * goc::kTab * 4)) ||
        (rc = dev_alloc((void**)&h->rowf_d, sum_ny * goc::kTab * 4)))
        return bail(rc);
    auto cleanup_tmp = [&]() { (void)hipFree(dh1_d); (void)hipFree(dh2_d); (void)hipFree(bmin_d); };
    if (hipMemcpy(h->h1_d, h1.data(), sum_nx * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dh1_d, dh1.data(), sum_nx * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->h2_d, h2.data(), sum_ny * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dh2_d, dh2.data(), sum_ny * 8, hipMemcpyHostToDevice) != hipSuccess) {
        cleanup_tmp();
        return bail(fail(GOC_EDEVICE, "metric upload failed"));
    }
    for (int r = 0; r < nruns; ++r) {
        RunDesc& d = h->runs[r];
        const int nbx = (d.nx + 255) / 256, nby = (d.ny + 255) / 256;
        (void)hipFree(bmin_d);
        bmin_d = nullptr;
        if (hipMalloc(&bmin_d, (nbx + nby) * 8) != hipSuccess) {
            cleanup_tmp();
            return bail(fail(GOC_ENOMEM, "hipMalloc failed"));
        }
        hipLaunchKernelGGL(goc::metric_kernel, dim3(nbx), dim3(256), 0, h->stream, h->h1_d + d.col_off,
                           dh1_d + d.col_off, h->th11_d + d.col_off, d.nx, bmin_d);
        hipLaunchKernelGGL(goc::metric_kernel, dim3(nby), dim3(256), 0, h->stream, h->h2_d + d.row_off,
                           dh2_d + d.row_off, h->th22_d + d.row_off, d.ny, bmin_d + nbx);
        std::vector<double> bm(nbx + nby);
        if (hipMemcpyAsync(bm.data(), bmin_d, (nbx + nby) * 8, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess) {
            cleanup_tmp();
            return bail(fail(GOC_EDEVICE, "metric precompute failed"));
        }
        // (a 2-D metric: the minimum over its node arrays)
        const double q = h->m2d ? h->m2[r].qmin : *std::min_element(bm.begin(), bm.end());
        h->q[r] = q;
        d.cs2 = q * q / 3.0;            // Sec. 3.2.1
        d.csm2 = d.cs2;                 // App. G: the same CFL-limited sound speed
        d.nu = d.cs2 * (1.0 / d.omega[4] - 0.5);
        d.zeta = d.cs2 * (1.0 / d.omega[3] - 0.5);
        d.eta = params[r].mhd ? d.csm2 * (params[r].tau_m - 0.5) : 0.0;
        // 16-bit storage scales per direction class: a tenth of the class's
        // rest-state magnitude maps to one, which keeps the deviations of
        // flows up to Mach 0.1 well inside the FP16 normal range
        const double c2 = d.cs2, r0 = d.rho0;
        const double mag[4] = {r0, 0.5 * r0 * c2, 0.5 * r0 * c2, 0.25 * r0 * c2 * c2};
        for (int k = 0; k < 4; ++k) d.sc[k] = 1.0 / std::max(mag[k] * 0.1, 1e-300);
        // D2Q5 deviations scale like h U B0 with U ~ Ma c_s
        d.scg = 1.0 / std::max(0.01 * std::fabs(d.B0) * std::sqrt(c2), 1e-12);
        goc::set_step_params(d);
        // column / row tables (FP64 and an FP32 copy, on the device)
        const double P0 = d.rho0 * d.cs2, W1B0 = 0.5 * d.csm2 * d.B0;
        hipLaunchKernelGGL(goc::table_kernel, dim3(nbx), dim3(256), 0, h->stream, h->h1_d + d.col_off,
                           h->th11_d + d.col_off, d.nx, d.bc_x == 0 ? 1 : 0, P0, W1B0,
                           h->col_d + d.col_off * goc::kTab, h->colf_d + d.col_off * goc::kTab);
        hipLaunchKernelGGL(goc::table_kernel, dim3(nby), dim3(256), 0, h->stream, h->h2_d + d.row_off,
                           h->th22_d + d.row_off, d.ny, d.bc_y == 0 ? 1 : 0, P0, W1B0,
                           h->row_d + d.row_off * goc::kTab, h->rowf_d + d.row_off * goc::kTab);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
            cleanup_tmp();
            return bail(fail(GOC_EDEVICE, "metric tables failed"));
        }
    }
    cleanup_tmp();
    if (h->m2d) {
        // 2-D metric planes (FP64 on the host, with their FP32 copy), face
        // values, and the node-moment buffer of the curvilinear step
        std::vector<double> met(met_elems), face(face_elems);
        for (int r = 0; r < nruns; ++r) {
            const RunDesc& d = h->runs[r];
            metric2d_planes(grid[r], h->m2[r], d.rho0 * d.cs2, met.data() + d.met_off);
            double* fr = face.data() + d.face_off;
            for (int j = 0; j < d.ny; ++j) {
                fr[2 * j] = h->m2[r].h1_lo[j];
                fr[2 * j + 1] = h->m2[r].h1_hi[j];
            }
            for (int i = 0; i < d.nx; ++i) {
                fr[2 * d.ny + 2 * i] = h->m2[r].h2_lo[i];
                fr[2 * d.ny + 2 * i + 1] = h->m2[r].h2_hi[i];
            }
        }
        std::vector<float> metf(met.begin(), met.end());
        if ((rc = dev_alloc((void**)&h->met_d, met_elems * 8)) || (rc = dev_alloc((void**)&h->metf_d, met_elems * 4)) ||
            (rc = dev_alloc((void**)&h->face_d, face_elems * 8)))
            return bail(rc);
        if (hipMemcpy(h->met_d, met.data(), met_elems * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(h->metf_d, metf.data(), met_elems * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(h->face_d, face.data(), face_elems * 8, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(GOC_EDEVICE, "2-D metric upload failed"));
    }
    {
        std::vector<double> th1(sum_nx), th2(sum_ny);
        if (hipMemcpy(th1.data(), h->th11_d, sum_nx * 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(th2.data(), h->th22_d, sum_ny * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return bail(fail(GOC_EDEVICE, "metric download failed"));
    }
    // run table, work list of the march and first tiles of the tiled step
    // (tiles of the smallest height built, so that every height fits)
    std::vector<int32_t> tile_first;
    bool overflow = false;
    h->tile_rows = goc::kTileRows[0];
    tile_table(h, tile_first, overflow);
    if (overflow) return bail(fail(GOC_EINVAL, "too many tiles in the launch"));
    h->tile_rows = goc::default_tile_rows((int)storage_bytes(storage));
    tile_table(h, tile_first, overflow);
    // non-temporal stores where one copy of the state exceeds half the
    // 256 MiB Infinity Cache (the autotuner times both)
    h->tile_nt = f_elems * sb + F_elems * fb > (size_t(128) << 20);
    h->total_tiles = tile_first[nruns];
    if ((rc = dev_alloc((void**)&h->runs_d, nruns * sizeof(RunDesc))) ||
        (rc = dev_alloc((void**)&h->block_run_d, block_run.size() * 4)) ||
        (rc = dev_alloc((void**)&h->tile_first_d, (nruns + 1) * 4)))
        return bail(rc);
    if (hipMemcpy(h->runs_d, h->runs.data(), nruns * sizeof(RunDesc), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->block_run_d, block_run.data(), block_run.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->tile_first_d, tile_first.data(), (nruns + 1) * 4, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(GOC_EDEVICE, "run table upload failed"));
    if ((rc = dev_alloc((void**)&h->step_ctr, 4))) return bail(rc);
    // reference tables of the 16-bit storage (zero: slots relative to the
    // rest state until the first refresh)
    h->ref_rows = sum_ny;
    if (scaled_storage(storage))
        for (int k = 0; k < 2; ++k) {
            if ((rc = dev_alloc((void**)&h->ref_d[k], h->ref_rows * goc::kRef * 4))) return bail(rc);
            if (hipMemsetAsync(h->ref_d[k], 0, h->ref_rows * goc::kRef * 4, h->stream) != hipSuccess)
                return bail(fail(GOC_EDEVICE, "reference table clear failed"));
        }
    // state pools
    for (int k = 0; k < 2; ++k) {
        if ((rc = dev_alloc(&h->f[k], f_elems * sb)) || (rc = dev_alloc(&h->F[k], F_elems * fb)))
            return bail(rc);
        if (hipMemsetAsync(h->f[k], 0, f_elems * sb, h->stream) != hipSuccess ||
            hipMemsetAsync(h->F[k], 0, F_elems * fb, h->stream) != hipSuccess)
            return bail(fail(GOC_EDEVICE, "state clear failed"));
    }
    *out = h;
    rc = goc_lbm_init(h, nullptr, nullptr, nullptr, 0);
    if (rc != GOC_OK) {
        *out = nullptr;
        return bail(rc);
    }
    return GOC_OK;
}

goc_lbm* check_handle(goc_lbm_t* h)
{
    if (!h) fail(GOC_EINVAL, "handle is NULL");
    return h;
}

// Allocate an FP64 device buffer of n doubles for host <-> device staging.
struct DevBuf {
    double* p = nullptr;
    ~DevBuf() { (void)hipFree(p); }
    int alloc(size_t n)
    {
        if (hipMalloc(&p, std::max<size_t>(n, 1) * 8) != hipSuccess)
            return fail(GOC_ENOMEM, "hipMalloc of %zu doubles failed", n);
        return GOC_OK;
    }
};

int init_run(goc_lbm* h, int run, const double* rho, const double* u1, const double* u2,
             const double* b1 = nullptr, const double* b2 = nullptr)
{
    const RunDesc& d = h->runs[run];
    return dispatch(h->storage, [&](auto tag) -> int {
        using S = decltype(tag);
        // write into the current input buffer
        auto pl = pools<S>(h, 1 - h->cur);
        hipLaunchKernelGGL(goc::init_kernel<S>, dim3(d.ny), dim3(256), 0, h->stream, h->runs_d, run, pl,
                           h->ref_d[0], rho, u1, u2, b1, b2);
        HIPOK(hipGetLastError());
        return GOC_OK;
    });
}

int gather_run(goc_lbm* h, int run, double* f, double* F, double* g, int on_device)
{
    const RunDesc& d = h->runs[run];
    const size_t N = (size_t)d.nx * d.ny;
    DevBuf bf, bF, bg;
    double *fd = f, *Fd = F, *gd = g;
    int rc;
    if (!on_device) {
        if ((rc = bf.alloc(9 * N)) || (rc = bF.alloc(2 * N))) return rc;
        fd = bf.p;
        Fd = bF.p;
        if (d.mhd && g) {
            if ((rc = bg.alloc(10 * N))) return rc;
            gd = bg.p;
        }
    }
    if (!d.mhd) gd = nullptr;
    dim3 grid, block;
    per_node_grid(d, grid, block);
    rc = dispatch(h->storage, [&](auto tag) -> int {
        using S = decltype(tag);
        auto pl = pools<S>(h, h->cur);
        hipLaunchKernelGGL(goc::gather_kernel<S>, grid, block, 0, h->stream, h->runs_d, run, pl, fd, Fd, gd);
        HIPOK(hipGetLastError());
        return GOC_OK;
    });
    if (rc) return rc;
    if (!on_device) {
        HIPOK(hipMemcpyAsync(f, fd, 9 * N * 8, hipMemcpyDeviceToHost, h->stream));
        HIPOK(hipMemcpyAsync(F, Fd, 2 * N * 8, hipMemcpyDeviceToHost, h->stream));
        if (gd) HIPOK(hipMemcpyAsync(g, gd, 10 * N * 8, hipMemcpyDeviceToHost, h->stream));
        HIPOK(hipStreamSynchronize(h->stream));
    }
    return GOC_OK;
}

int fields_run(goc_lbm* h, int run, double* rho, double* u, double* B, int on_device)
{
    const RunDesc& d = h->runs[run];
    const size_t N = (size_t)d.nx * d.ny;
    DevBuf br, bu, bB;
    double *rd = rho, *ud = u, *Bd = d.mhd ? B : nullptr;
    int rc;
    if (!on_device) {
        if (rho && (rc = br.alloc(N))) return rc;
        if (u && (rc = bu.alloc(2 * N))) return rc;
        if (Bd && (rc = bB.alloc(2 * N))) return rc;
        rd = rho ? br.p : nullptr;
        ud = u ? bu.p : nullptr;
        Bd = Bd ? bB.p : nullptr;
    }
    dim3 grid, block;
    per_node_grid(d, grid, block);
    rc = dispatch(h->storage, [&](auto tag) -> int {
        using S = decltype(tag);
        auto pl = pools<S>(h, h->cur);
        hipLaunchKernelGGL(goc::fields_kernel<S>, grid, block, 0, h->stream, h->runs_d, run, pl, rd, ud, Bd);
        HIPOK(hipGetLastError());
        return GOC_OK;
    });
    if (rc) return rc;
    if (!on_device) {
        if (rho) HIPOK(hipMemcpyAsync(rho, rd, N * 8, hipMemcpyDeviceToHost, h->stream));
        if (u) HIPOK(hipMemcpyAsync(u, ud, 2 * N * 8, hipMemcpyDeviceToHost, h->stream));
        if (Bd) HIPOK(hipMemcpyAsync(B, Bd, 2 * N * 8, hipMemcpyDeviceToHost, h->stream));
        HIPOK(hipStreamSynchronize(h->stream));
    }
    return GOC_OK;
}

// Work-groups of the diagnostics' first pass over a run (each strides over
// the nodes; at most goc::kDiagBlocks).
int diag_blocks(const RunDesc& d)
{
    const int64_t N = (int64_t)d.nx * d.ny;
    return (int)std::min<int64_t>((N + 255) / 256, goc::kDiagBlocks);
}

// The two passes of the diagnostics of run `run` into out_dev (8 doubles,
// device), with `part` (diag_blocks doubles x goc::kDiag) as the partials.
int launch_diag(goc_lbm* h, int run, double* part, double* out_dev)
{
    const int nb = diag_blocks(h->runs[run]);
    int rc = dispatch(h->storage, [&](auto tag) -> int {
        using S = decltype(tag);
        auto pl = pools<S>(h, h->cur);
        hipLaunchKernelGGL(goc::diag_kernel<S>, dim3(nb), dim3(256), 0, h->stream, h->runs_d, run, pl, part);
        HIPOK(hipGetLastError());
        return GOC_OK;
    });
    if (rc) return rc;
    hipLaunchKernelGGL(goc::diag_final_kernel, dim3(1), dim3(256), 0, h->stream, part, nb, h->runs[run].nx,
                       out_dev);
    HIPOK(hipGetLastError());
    return GOC_OK;
}

// Diagnostics of run `run` into the host array out[8] (the partials in a
// buffer of the handle, allocated on first use).
int diag_run(goc_lbm* h, int run, double out[8])
{
    const int nb = diag_blocks(h->runs[run]);
    if (nb > h->diag_cap) {
        (void)hipFree(h->diag_part);
        h->diag_part = nullptr;
        if (hipMalloc(&h->diag_part, (size_t)nb * goc::kDiag * 8) != hipSuccess)
            return fail(GOC_ENOMEM, "diagnostics scratch allocation failed");
        h->diag_cap = nb;
    }
    if (!h->diag_out && hipMalloc(&h->diag_out, 8 * 8) != hipSuccess)
        return fail(GOC_ENOMEM, "diagnostics allocation failed");
    if (int rc = launch_diag(h, run, h->diag_part, h->diag_out)) return rc;
    HIPOK(hipMemcpyAsync(out, h->diag_out, 8 * 8, hipMemcpyDeviceToHost, h->stream));
    HIPOK(hipStreamSynchronize(h->stream));
    return GOC_OK;
}

// Scratch of goc_lbm_diagnostics_noalloc: room for the partials of the
// diagnostics' first pass at its largest grid (goc::kDiagBlocks x
// goc::kDiag doubles, 229 KB), in every device's memory from the library's
// loading until the process ends.  Host code never uses the name itself
// (a host-side stand-in): each device's copy is reached through the address
// scratch_on returns.
__device__ __align__(256) double scratch[goc::kDiagBlocks * goc::kDiag];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch` on each device

// The address of `scratch` on the current device `device`, looked up with
// that device current on its first use and kept.
int scratch_on(int device, double** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return fail(GOC_EDEVICE, "device %d beyond %d", device, kMaxDevices);
    if (!g_scratch_dev[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GOC_EDEVICE, "hipGetSymbolAddress of the diagnostics scratch failed: %s",
                        hipGetErrorString(e));
        g_scratch_dev[device] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[device];
    return GOC_OK;
}

int capture_graph(goc_lbm* h, int parity)
{
    hipGraph_t g = nullptr;
    const int saved = h->cur;
    h->cur = parity;
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        h->cur = saved;
        return fail(GOC_EDEVICE, "graph capture could not start (the stream must not be the NULL stream)");
    }
    int rc = GOC_OK;
    for (int s = 0; s < kGraphSteps && rc == GOC_OK; ++s) {
        rc = launch_step(h, s, scaled_storage(h->storage) && s == 0);
        h->cur ^= 1;
    }
    if (rc == GOC_OK) rc = counter_op(h, kGraphSteps, 1);
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    h->cur = saved;
    if (rc != GOC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(GOC_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&h->graph[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(GOC_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    return GOC_OK;
}

}  // namespace

// =================================================================== C ABI ==
extern "C" {

const char* goc_lbm_last_error(void) { return g_err.c_str(); }

int goc_lbm_derive(goc_grid* grid, const goc_metric* metric, const goc_physics* phys, goc_params* out)
{
    int rc;
    if ((rc = check_grid(grid)) != GOC_OK) return rc;
    if (!metric || !phys || !out) return fail(GOC_EINVAL, "NULL metric, physics or output");
    Metric1D mx, my;
    if ((rc = build_metric(*grid, *metric, mx, my)) != GOC_OK) return rc;
    double q = std::min(*std::min_element(mx.h.begin(), mx.h.end()), *std::min_element(my.h.begin(), my.h.end()));
    if (is_2d(*metric)) {
        Metric2D m2;
        if ((rc = build_metric2d(*grid, *metric, m2)) != GOC_OK) return rc;
        q = m2.qmin;
    }
    const double cs2 = q * q / 3.0;
    const double rho0 = phys->rho0 > 0 ? phys->rho0 : 1.0;
    goc_params p;
    std::memset(&p, 0, sizeof(p));
    for (int k = 0; k < 9; ++k) p.omega[k] = 1.0;
    p.rho0 = rho0;
    p.gi_terms = 1;
    p.lid_corners = 1;
    p.mu_m = phys->mu_m > 0 ? phys->mu_m : 1.0;
    p.tau_m = 1.0;
    double nu = 0.0;
    switch (phys->flow) {
    case GOC_FLOW_CHANNEL: {
        if (!(phys->tau > 0.5)) return fail(GOC_EINVAL, "channel flow needs tau > 1/2");
        nu = cs2 * (phys->tau - 0.5);
        const double half = 0.5 * grid->ny;
        const double U = phys->Re * nu / half;
        p.F_ext[0] = 2.0 * nu * U * rho0 / (half * half);
        break;
    }
    case GOC_FLOW_CAVITY: {
        if (!(phys->Re > 0)) return fail(GOC_EINVAL, "cavity flow needs Re > 0");
        double ul = phys->u_lid > 0 ? phys->u_lid : phys->Ma * std::sqrt(cs2);
        if (!(ul > 0)) return fail(GOC_EINVAL, "cavity flow needs u_lid > 0 or Ma > 0");
        nu = ul * grid->nx / phys->Re;
        if (!(phys->u_lid > 0) && phys->tau_max > 0.5 && nu > cs2 * (phys->tau_max - 0.5)) {
            nu = cs2 * (phys->tau_max - 0.5);     // relaxation-time cap, Re kept
            ul = nu * phys->Re / grid->nx;
        }
        grid->u_wall_hi = ul;
        break;
    }
    case GOC_FLOW_HARTMANN: {
        if (!(phys->Re > 0) || !(phys->Pm > 0) || !(phys->Ma > 0))
            return fail(GOC_EINVAL, "Hartmann flow needs Re, Pm, Ma > 0");
        const double H = 0.5 * grid->ny;
        double Uc = phys->Ma * std::sqrt(cs2);
        nu = Uc * H / phys->Re;
        if (phys->tau_max > 0.5 && nu > cs2 * (phys->tau_max - 0.5)) {
            nu = cs2 * (phys->tau_max - 0.5);     // relaxation-time cap, Re kept
            Uc = nu * phys->Re / H;
        }
        const double eta = nu / phys->Pm;
        const double sigma = 1.0 / (eta * p.mu_m);
        const double Ha = phys->Ha;
        p.B0 = Ha > 0 ? Ha / (H * std::sqrt(sigma / (rho0 * nu))) : 0.0;
        const double shape = Ha > 0 ? (1.0 - 1.0 / std::cosh(Ha)) / (Ha * std::tanh(Ha)) : 0.5;
        p.F_ext[0] = Uc * rho0 * nu / (H * H * shape);
        p.mhd = 1;
        p.tau_m = eta / cs2 + 0.5;
        break;
    }
    case GOC_FLOW_FREE:
        if (!(phys->tau > 0.5)) return fail(GOC_EINVAL, "free flow needs tau > 1/2");
        nu = cs2 * (phys->tau - 0.5);
        p.F_ext[0] = phys->F_ext[0];
        p.F_ext[1] = phys->F_ext[1];
        break;
    default:
        return fail(GOC_EINVAL, "unknown flow kind %d", phys->flow);
    }
    if (!(nu > 0)) return fail(GOC_EINVAL, "derived viscosity %g is not positive", nu);
    p.omega[4] = p.omega[5] = 1.0 / (nu / cs2 + 0.5);
    *out = p;
    return GOC_OK;
}

int goc_lbm_create(goc_lbm_t** out, const goc_grid* grid, const goc_metric* metric, const goc_params* params,
                   int32_t storage, void* stream)
{
    return create_impl(out, 1, grid, metric, params, storage, stream);
}

int goc_lbm_create_batch(goc_lbm_t** out, int32_t nruns, const goc_grid* grid, const goc_metric* metric,
                         const goc_params* params, int32_t storage, void* stream)
{
    return create_impl(out, nruns, grid, metric, params, storage, stream);
}

int32_t goc_lbm_num_runs(const goc_lbm_t* h) { return h ? h->nruns : 0; }

void goc_lbm_destroy(goc_lbm_t* h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
}

namespace {
// Fields of one run (all five given or B NULL); the caller resets the step.
int init_fields(goc_lbm* h, int run, const double* rho, const double* u1, const double* u2, const double* b1,
                const double* b2, int32_t on_device)
{
    const RunDesc& d = h->runs[run];
    const size_t N = (size_t)d.nx * d.ny;
    const double* src[5] = {rho, u1, u2, b1, b2};
    const double* dev[5] = {rho, u1, u2, b1, b2};
    DevBuf buf[5];
    if (!on_device) {
        for (int k = 0; k < 5; ++k) {
            if (!src[k]) continue;
            if (int rc = buf[k].alloc(N)) return rc;
            HIPOK(hipMemcpyAsync(buf[k].p, src[k], N * 8, hipMemcpyHostToDevice, h->stream));
            dev[k] = buf[k].p;
        }
    }
    int rc = init_run(h, run, dev[0], dev[1], dev[2], dev[3], dev[4]);
    if (rc) return rc;
    HIPOK(hipStreamSynchronize(h->stream));
    return GOC_OK;
}

int check_fields(const goc_lbm* h, int run, const double* rho, const double* u1, const double* u2,
                 const double* b1, const double* b2)
{
    if (!(rho && u1 && u2)) return fail(GOC_EINVAL, "init needs all of rho, u1, u2");
    if ((b1 != nullptr) != (b2 != nullptr)) return fail(GOC_EINVAL, "init needs both of b1, b2 or neither");
    if (b1 && !h->runs[run].mhd) return fail(GOC_EINVAL, "b1, b2 given for a run without MHD");
    return GOC_OK;
}
}  // namespace

int goc_lbm_init_run(goc_lbm_t* h, int32_t run, const double* rho, const double* u1, const double* u2,
                     const double* b1, const double* b2, int32_t on_device)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (run < 0 || run >= h->nruns) return fail(GOC_EINVAL, "run %d outside [0, %d)", run, h->nruns);
    if (int rc = check_fields(h, run, rho, u1, u2, b1, b2)) return rc;
    if (int rc = init_fields(h, run, rho, u1, u2, b1, b2, on_device)) return rc;
    h->ref_base = h->step;   // (16-bit storage: refresh the reference table next)
    return GOC_OK;
}

int goc_lbm_init_mhd(goc_lbm_t* h, const double* rho, const double* u1, const double* u2, const double* b1,
                     const double* b2, int32_t on_device)
{
    if (!check_handle(h)) return GOC_EINVAL;
    const bool given = rho || u1 || u2;
    if (!given && (b1 || b2)) return fail(GOC_EINVAL, "b1, b2 need rho, u1, u2 too");
    if (given) {
        if (int rc = check_fields(h, 0, rho, u1, u2, b1, b2)) return rc;
        if (h->nruns != 1) return fail(GOC_EINVAL, "field initialisation of a batch is per run (goc_lbm_init_run)");
    }
    // write into the input buffer: kernels write to "out" of pools(1 - cur)
    if (!given) {
        for (int r = 0; r < h->nruns; ++r) {
            int rc = init_run(h, r, nullptr, nullptr, nullptr);
            if (rc) return rc;
        }
    } else {
        if (int rc = init_fields(h, 0, rho, u1, u2, b1, b2, on_device)) return rc;
    }
    h->step = 0;
    h->watch_last = 0;
    h->ref_base = 0;
    if (int rc = counter_op(h, 0, 0)) return rc;
    HIPOK(hipStreamSynchronize(h->stream));
    return GOC_OK;
}

int goc_lbm_init(goc_lbm_t* h, const double* rho, const double* u1, const double* u2, int32_t on_device)
{
    return goc_lbm_init_mhd(h, rho, u1, u2, nullptr, nullptr, on_device);
}

int goc_lbm_step(goc_lbm_t* h, int64_t n)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (n < 0) return fail(GOC_EINVAL, "negative step count");
    // 16-bit storage: an initialisation forms the reference table from the
    // initial state; the steps refresh it from the state after the first
    // step (whose collision adds the lagged force) and then every kGraphSteps
    // steps (steps ref_base + 1 + m kGraphSteps), which is where its graph
    // blocks start: a block refreshes on its first step.  Graph blocks and
    // single launches therefore refresh on the same steps.
    const bool scaled = scaled_storage(h->storage);
    const int64_t b0 = h->ref_base + 1;
    auto block_start = [&](int64_t s) { return !scaled || (s >= b0 && (s - b0) % kGraphSteps == 0); };
    auto refresh_at = [&](int64_t s) { return scaled && s >= b0 && (s - b0) % kGraphSteps == 0; };
    while (n > 0) {
        const int64_t chunk = n;
        int64_t done = 0;
        while (done < chunk) {
            const int64_t s = h->step + done;
            // whole graph blocks when a capturable stream is in use
            if (h->stream && block_start(s) && chunk - done >= kGraphSteps) {
                if (!h->graph[h->cur]) {
                    int rc = capture_graph(h, h->cur);
                    if (rc) return rc;
                }
                HIPOK(hipGraphLaunch(h->graph[h->cur], h->stream));
                done += kGraphSteps;   // an even count: parity unchanged
                continue;
            }
            // single launches, in pieces that keep k small (with graphs: up
            // to the next block start)
            int64_t piece = std::min<int64_t>(chunk - done, 4096);
            if (h->stream && !block_start(s)) {
                const int64_t next = s < b0 ? b0 : b0 + ((s - b0) / kGraphSteps + 1) * kGraphSteps;
                piece = std::min<int64_t>(piece, next - s);
            }
            for (int t = 0; t < (int)piece; ++t) {
                int rc = launch_step(h, t, refresh_at(s + t));
                if (rc) return rc;
                h->cur ^= 1;
            }
            int rc = counter_op(h, (uint32_t)piece, 1);
            if (rc) return rc;
            done += piece;
        }
        h->step += chunk;
        n -= chunk;
    }
    // the watchdog: at the return of a call that completes at least
    // `watchdog` steps since the last check, every run's non-finite count
    if (h->watchdog > 0 && h->step - h->watch_last >= h->watchdog) {
        h->watch_last = h->step;
        for (int r = 0; r < h->nruns; ++r) {
            double o[8];
            int rc = diag_run(h, r, o);
            if (rc) return rc;
            if (o[7] > 0)
                return fail(GOC_EUNSTABLE, "run %d: %g non-finite values at step %lld", r, o[7], (long long)h->step);
        }
    }
    return GOC_OK;
}

int goc_lbm_set_launch(goc_lbm_t* h, double waves_per_cu)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (waves_per_cu == 0.0) {
        if (h->m2d) return GOC_OK;   // always tiled
        return use_tiled(h);
    }
    if (h->m2d) return fail(GOC_EINVAL, "a run on a 2-D metric has only the tiled step (waves_per_cu 0)");
    if (scaled_storage(h->storage))
        return fail(GOC_EINVAL, "16-bit storage has only the tiled step (waves_per_cu 0)");
    if (!(waves_per_cu >= 0.5 && waves_per_cu <= 1024.0))
        return fail(GOC_EINVAL, "waves_per_cu %g outside [0.5, 1024]", waves_per_cu);
    return apply_plan(h, waves_per_cu);
}

int goc_lbm_launch_info(const goc_lbm_t* h, double out[6])
{
    if (!h || !out) return fail(GOC_EINVAL, "NULL handle or output");
    int64_t rows = 0, segs = 0, strips = 0;
    for (const RunDesc& d : h->runs) {
        rows += (int64_t)d.ny * d.strips;
        segs += (int64_t)d.segs * d.strips;
        strips += d.strips;
    }
    if (h->m2d || h->tiled) {
        const int ty = h->tile_rows, tw = h->tile_cols;
        int64_t tiles = 0, cols = 0;
        for (const RunDesc& d : h->runs) {
            const int64_t gx = (d.nx + tw - 1) / tw;
            tiles += gx * ((d.ny + ty - 1) / ty);
            cols += gx;
        }
        out[0] = 0.0;
        out[1] = (double)tiles;
        out[2] = ty;
        out[3] = (double)cols;
        out[4] = h->tile_nt ? 1.0 : 0.0;
        out[5] = tw;
        return GOC_OK;
    }
    out[0] = h->waves_per_cu;
    out[1] = h->total_blocks;
    out[2] = segs ? double(rows) / double(segs) : 0.0;
    out[3] = (double)strips;
    out[4] = 0.0;
    out[5] = goc::kWave;
    return GOC_OK;
}

int goc_lbm_set_tile_shape(goc_lbm_t* h, int32_t cols, int32_t rows, int32_t nontemporal)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (!tile_shape_built(cols, rows, h->storage, h->m2d))
        return fail(GOC_EINVAL, "tile shape %d x %d: 64 x 4, 8 or 16 (FP64: 4 or 8), or 128 x 4 on straight grids",
                    cols, rows);
    if (nontemporal != 0 && nontemporal != 1) return fail(GOC_EINVAL, "nontemporal must be 0 or 1");
    return use_tiled(h, cols, rows, nontemporal);
}

int goc_lbm_set_tile(goc_lbm_t* h, int32_t rows, int32_t nontemporal)
{
    return goc_lbm_set_tile_shape(h, goc::kTileX, rows, nontemporal);
}

int goc_lbm_tune(goc_lbm_t* h, int32_t trial_steps, double out[4])
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (!out) return fail(GOC_EINVAL, "out is NULL");
    if (trial_steps < 1 || trial_steps > 10000) return fail(GOC_EINVAL, "trial_steps %d outside [1, 10000]", trial_steps);
    static const double cand[] = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512};
    struct Ev {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Ev() { for (auto x : e) if (x) (void)hipEventDestroy(x); }
    } ev;
    HIPOK(hipEventCreate(&ev.e[0]));
    HIPOK(hipEventCreate(&ev.e[1]));
    // The trials step the state as a run does, each launch reading what the
    // last one wrote (a trial that read the same buffer every time would find
    // part of it still in the Infinity Cache, which a run never does, and
    // favour the forms that keep it there); the state is copied first and
    // put back afterwards, so the run does not change.  A candidate is
    // (waves_per_cu, tile rows, store policy): waves_per_cu 0 is the tiled
    // step with that tile height, a positive one the march with that plan.
    const size_t sb = storage_bytes(h->storage), fb = force_bytes(h->storage);
    const size_t bytes[2] = {h->f_elems * sb, h->F_elems * fb};
    void* const* bufs[2] = {h->f, h->F};
    struct Saved {
        void* p[2] = {nullptr, nullptr};
        ~Saved() { for (auto x : p) if (x) (void)hipFree(x); }
    } saved;
    const int cur0 = h->cur;
    for (int k = 0; k < 2; ++k) {
        if (!bytes[k]) continue;
        if (hipMalloc(&saved.p[k], bytes[k]) != hipSuccess) {
            saved.p[k] = nullptr;
            (void)hipStreamSynchronize(h->stream);   // (copies into the earlier buffers may be in flight)
            return fail(GOC_ENOMEM, "tuner: no device memory for a copy of the state (%zu bytes)", bytes[k]);
        }
        HIPOK(hipMemcpyAsync(saved.p[k], bufs[k][cur0], bytes[k], hipMemcpyDeviceToDevice, h->stream));
    }
    auto restore = [&]() -> int {
        h->cur = cur0;
        for (int k = 0; k < 2; ++k)
            if (bytes[k])
                HIPOK(hipMemcpyAsync(bufs[k][cur0], saved.p[k], bytes[k], hipMemcpyDeviceToDevice, h->stream));
        HIPOK(hipStreamSynchronize(h->stream));
        return GOC_OK;
    };
    struct Cand {
        double w;    // 0: the tiled step, > 0: the march with this plan
        int rows;    // tile height
        int nt;      // non-temporal stores (tiled step)
        int cols;    // tile width
    };
    auto select = [&](const Cand& c) -> int {
        return c.w == 0.0 ? use_tiled(h, c.cols, c.rows, c.nt) : apply_plan(h, c.w);
    };
    auto time_form = [&](const Cand& c, int steps, double& us) -> int {
        int rc = select(c);
        if (rc) return rc;
        if ((rc = launch_step(h, 0))) return rc;
        h->cur ^= 1;
        HIPOK(hipEventRecord(ev.e[0], h->stream));
        for (int s = 0; s < steps; ++s) {
            if ((rc = launch_step(h, s))) return rc;
            h->cur ^= 1;
        }
        HIPOK(hipEventRecord(ev.e[1], h->stream));
        HIPOK(hipEventSynchronize(ev.e[1]));
        float ms = 0.0f;
        HIPOK(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
        us = 1e3 * ms / steps;
        return GOC_OK;
    };
    // the tiled step at every tile shape, with and without non-temporal
    // stores, then (straight FP64 / FP32 runs) the march at every plan
    const bool march = tile_eligible(h) && !scaled_storage(h->storage);
    const Cand prev = {(h->m2d || h->tiled) ? 0.0 : h->waves_per_cu, h->tile_rows, h->tile_nt ? 1 : 0,
                       h->tile_cols};
    std::vector<Cand> cands;
    for (int rows : goc::kTileRows)
        if (tile_shape_built(goc::kTileX, rows, h->storage, h->m2d))
            for (int nt = 0; nt < 2; ++nt) cands.push_back({0.0, rows, nt, goc::kTileX});
    if (tile_shape_built(goc::kTileXWide, goc::kTileRowsWide, h->storage, h->m2d))
        for (int nt = 0; nt < 2; ++nt) cands.push_back({0.0, goc::kTileRowsWide, nt, goc::kTileXWide});
    if (march)
        for (double w : cand) cands.push_back({w, prev.rows, prev.nt, prev.cols});
    double best_us = 1e300, prev_us = -1.0;
    Cand best = prev;
    std::vector<double> times;
    for (const auto& c : cands) {
        double us = 0.0;
        if (int rc = time_form(c, trial_steps, us)) {
            (void)restore();
            return rc;
        }
        times.push_back(us);
        if (c.w == prev.w && (prev.w != 0.0 || (c.rows == prev.rows && c.nt == prev.nt && c.cols == prev.cols)))
            prev_us = us;
        if (us < best_us) {
            best_us = us;
            best = c;
        }
    }
    // the close finishers (within 5 % of the fastest) once more with three
    // times the steps: one short timing can swap forms that lie within a few
    // percent of each other
    const int steps2 = std::min(10000, 3 * trial_steps);
    double best2 = 1e300;
    for (size_t c = 0; c < cands.size(); ++c) {
        if (times[c] > 1.05 * best_us) continue;
        double us = 0.0;
        if (int rc = time_form(cands[c], steps2, us)) {
            (void)restore();
            return rc;
        }
        if (us < best2) {
            best2 = us;
            best = cands[c];
        }
    }
    if (int rc = restore()) return rc;
    if (int rc = select(best)) return rc;
    out[0] = best.w;
    out[1] = best2;
    out[2] = prev_us;
    out[3] = (double)cands.size();
    return GOC_OK;
}

int goc_lbm_set_watchdog(goc_lbm_t* h, int64_t every)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (every < 0) return fail(GOC_EINVAL, "negative watchdog interval");
    h->watchdog = every;
    h->watch_last = h->step;
    return GOC_OK;
}

int goc_lbm_moments_run(goc_lbm_t* h, int32_t run, double* rho, double* u, double* B, int32_t on_device)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (run < 0 || run >= h->nruns) return fail(GOC_EINVAL, "run %d out of range", run);
    return fields_run(h, run, rho, u, B, on_device);
}

int goc_lbm_moments(goc_lbm_t* h, double* rho, double* u, double* B, int32_t on_device)
{
    return goc_lbm_moments_run(h, 0, rho, u, B, on_device);
}

int goc_lbm_diagnostics_run(goc_lbm_t* h, int32_t run, double out[8])
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (!out) return fail(GOC_EINVAL, "out is NULL");
    if (run < 0 || run >= h->nruns) return fail(GOC_EINVAL, "run %d outside [0, %d)", run, h->nruns);
    return diag_run(h, run, out);
}

int goc_lbm_diagnostics(goc_lbm_t* h, double out[8]) { return goc_lbm_diagnostics_run(h, 0, out); }

int goc_lbm_diagnostics_noalloc(goc_lbm_t* h, int32_t run, double* out_dev)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (!out_dev) return fail(GOC_EINVAL, "out_dev is NULL");
    if (run < 0 || run >= h->nruns) return fail(GOC_EINVAL, "run %d outside [0, %d)", run, h->nruns);
    int device = -1;
    HIPOK(hipGetDevice(&device));
    if (device != h->device)
        return fail(GOC_EINVAL, "current device %d is not the handle's device %d", device, h->device);
    if (diag_blocks(h->runs[run]) > goc::kDiagBlocks)   // (the first pass strides: never true)
        return fail(GOC_EINVAL, "diagnostics of run %d need more than the %d partials of the scratch", run,
                    goc::kDiagBlocks);
    double* part = nullptr;
    if (int rc = scratch_on(device, &part)) return rc;
    return launch_diag(h, run, part, out_dev);
}

int goc_lbm_get_populations_run(goc_lbm_t* h, int32_t run, double* f, double* F, double* g, int32_t on_device)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (run < 0 || run >= h->nruns) return fail(GOC_EINVAL, "run %d out of range", run);
    if (!f || !F) return fail(GOC_EINVAL, "f and F are required");
    return gather_run(h, run, f, F, g, on_device);
}

int goc_lbm_get_populations(goc_lbm_t* h, double* f, double* F, double* g, int32_t on_device)
{
    return goc_lbm_get_populations_run(h, 0, f, F, g, on_device);
}

int goc_lbm_set_populations(goc_lbm_t* h, const double* f, const double* F, const double* g, int32_t on_device)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (!f || !F) return fail(GOC_EINVAL, "f and F are required");
    const RunDesc& d = h->runs[0];
    if (d.mhd && !g) return fail(GOC_EINVAL, "MHD run needs g");
    const size_t N = (size_t)d.nx * d.ny;
    DevBuf bf, bF, bg;
    const double *fd = f, *Fd = F, *gd = d.mhd ? g : nullptr;
    int rc;
    if (!on_device) {
        if ((rc = bf.alloc(9 * N)) || (rc = bF.alloc(2 * N))) return rc;
        HIPOK(hipMemcpyAsync(bf.p, f, 9 * N * 8, hipMemcpyHostToDevice, h->stream));
        HIPOK(hipMemcpyAsync(bF.p, F, 2 * N * 8, hipMemcpyHostToDevice, h->stream));
        fd = bf.p;
        Fd = bF.p;
        if (gd) {
            if ((rc = bg.alloc(10 * N))) return rc;
            HIPOK(hipMemcpyAsync(bg.p, g, 10 * N * 8, hipMemcpyHostToDevice, h->stream));
            gd = bg.p;
        }
    }
    rc = dispatch(h->storage, [&](auto tag) -> int {
        using S = decltype(tag);
        auto pl = pools<S>(h, 1 - h->cur);   // out = current input buffer
        hipLaunchKernelGGL(goc::scatter_kernel<S>, dim3(d.ny), dim3(256), 0, h->stream, h->runs_d, 0, pl,
                           h->ref_d[0], fd, Fd, gd);
        HIPOK(hipGetLastError());
        return GOC_OK;
    });
    if (rc) return rc;
    HIPOK(hipStreamSynchronize(h->stream));
    h->ref_base = h->step;
    return GOC_OK;
}

namespace {
// Checkpoint blob: this header, then per run (nx, ny, mhd) as int32, then
// the reference table of the 16-bit storage, the slot pool (with the D2Q5
// slots of MHD runs in its rows) and the lagged force, each as the raw
// device bytes.
struct StateHeader {
    char magic[8];
    int32_t version, storage, nruns, mhd;
    int64_t step, f_bytes, F_bytes, ref_bytes, ref_base;
};
constexpr int32_t kStateVersion = 3;

StateHeader state_header(const goc_lbm* h)
{
    const size_t sb = storage_bytes(h->storage), fb = force_bytes(h->storage);
    StateHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    std::memcpy(hd.magic, "GOCLBM01", 8);
    hd.version = kStateVersion;
    hd.storage = h->storage;
    hd.nruns = h->nruns;
    hd.mhd = h->any_mhd;
    hd.step = h->step;
    hd.f_bytes = h->f_elems * sb;
    hd.F_bytes = h->F_elems * fb;
    hd.ref_bytes = scaled_storage(h->storage) ? h->ref_rows * goc::kRef * 4 : 0;
    hd.ref_base = h->ref_base;
    return hd;
}

void run_shapes(const goc_lbm* h, std::vector<int32_t>& v)
{
    v.clear();
    for (const RunDesc& d : h->runs) {
        v.push_back(d.nx);
        v.push_back(d.ny);
        v.push_back(d.mhd);
    }
}
}  // namespace

int goc_lbm_get_state(goc_lbm_t* h, void* buf, size_t* bytes)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (!bytes) return fail(GOC_EINVAL, "bytes is NULL");
    const StateHeader hd = state_header(h);
    std::vector<int32_t> shapes;
    run_shapes(h, shapes);
    const size_t sh_bytes = shapes.size() * 4;
    const size_t need = sizeof(hd) + sh_bytes + hd.ref_bytes + hd.f_bytes + hd.F_bytes;
    if (!buf) {
        *bytes = need;
        return GOC_OK;
    }
    if (*bytes < need) return fail(GOC_EINVAL, "state buffer of %zu bytes, need %zu", *bytes, need);
    char* p = static_cast<char*>(buf);
    std::memcpy(p, &hd, sizeof(hd));
    p += sizeof(hd);
    std::memcpy(p, shapes.data(), sh_bytes);
    p += sh_bytes;
    if (hd.ref_bytes) HIPOK(hipMemcpyAsync(p, h->ref_d[0], hd.ref_bytes, hipMemcpyDeviceToHost, h->stream));
    p += hd.ref_bytes;
    HIPOK(hipMemcpyAsync(p, h->f[h->cur], hd.f_bytes, hipMemcpyDeviceToHost, h->stream));
    HIPOK(hipMemcpyAsync(p + hd.f_bytes, h->F[h->cur], hd.F_bytes, hipMemcpyDeviceToHost, h->stream));
    HIPOK(hipStreamSynchronize(h->stream));
    *bytes = need;
    return GOC_OK;
}

int goc_lbm_set_state(goc_lbm_t* h, const void* buf, size_t bytes)
{
    if (!check_handle(h)) return GOC_EINVAL;
    if (!buf) return fail(GOC_EINVAL, "buf is NULL");
    const StateHeader mine = state_header(h);
    std::vector<int32_t> shapes;
    run_shapes(h, shapes);
    const size_t sh_bytes = shapes.size() * 4;
    if (bytes < sizeof(StateHeader)) return fail(GOC_ESTATE, "state blob of %zu bytes is shorter than its header", bytes);
    StateHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (std::memcmp(hd.magic, "GOCLBM01", 8) != 0 || hd.version != kStateVersion || hd.storage != h->storage ||
        hd.nruns != h->nruns || hd.mhd != mine.mhd)
        return fail(GOC_ESTATE, "state blob does not match this run (magic, version, storage, run count or MHD)");
    if (hd.f_bytes != mine.f_bytes || hd.F_bytes != mine.F_bytes || hd.ref_bytes != mine.ref_bytes)
        return fail(GOC_ESTATE, "state blob sizes (slots %lld, force %lld, reference %lld bytes) do not "
                    "match this run's (%lld, %lld, %lld)", (long long)hd.f_bytes, (long long)hd.F_bytes,
                    (long long)hd.ref_bytes, (long long)mine.f_bytes, (long long)mine.F_bytes,
                    (long long)mine.ref_bytes);
    const size_t need = sizeof(hd) + sh_bytes + hd.ref_bytes + hd.f_bytes + hd.F_bytes;
    if (bytes != need) return fail(GOC_ESTATE, "state blob of %zu bytes, this run needs %zu", bytes, need);
    const char* p = static_cast<const char*>(buf) + sizeof(hd);
    if (std::memcmp(p, shapes.data(), sh_bytes) != 0)
        return fail(GOC_ESTATE, "state blob of other grid sizes or MHD flags than this run's");
    if (hd.step < 0 || hd.ref_base < 0 || hd.ref_base > hd.step)
        return fail(GOC_ESTATE, "state blob with an inconsistent step count");
    p += sh_bytes;
    if (hd.ref_bytes) HIPOK(hipMemcpyAsync(h->ref_d[0], p, hd.ref_bytes, hipMemcpyHostToDevice, h->stream));
    p += hd.ref_bytes;
    HIPOK(hipMemcpyAsync(h->f[h->cur], p, hd.f_bytes, hipMemcpyHostToDevice, h->stream));
    HIPOK(hipMemcpyAsync(h->F[h->cur], p + hd.f_bytes, hd.F_bytes, hipMemcpyHostToDevice, h->stream));
    h->step = hd.step;
    h->watch_last = hd.step;
    h->ref_base = hd.ref_base;
    if (int rc = counter_op(h, (uint32_t)hd.step, 0)) return rc;
    HIPOK(hipStreamSynchronize(h->stream));
    return GOC_OK;
}

int goc_lbm_derived_run(const goc_lbm_t* h, int32_t run, double out[16])
{
    if (!h) return fail(GOC_EINVAL, "handle is NULL");
    if (!out) return fail(GOC_EINVAL, "out is NULL");
    if (run < 0 || run >= h->nruns) return fail(GOC_EINVAL, "run %d outside [0, %d)", run, h->nruns);
    const RunDesc& d = h->runs[run];
    const double sb = (double)storage_bytes(h->storage), fb = (double)force_bytes(h->storage);
    out[0] = d.cs2;
    out[1] = d.nu;
    out[2] = d.zeta;
    out[3] = h->q[run];
    out[4] = d.csm2;
    out[5] = d.eta;
    out[6] = d.tau_m;
    out[7] = d.B0;
    out[8] = d.Fx1;
    out[9] = d.Fx2;
    out[10] = d.hw_lo;
    out[11] = d.hw_hi;
    out[12] = (double)h->step;
    // algorithmic bytes per node update: populations and lagged force read
    // and written, the D2Q5 slots for MHD, the metric planes of a 2-D run
    out[13] = 2.0 * (9.0 * sb + 2.0 * fb + (d.mhd ? 10.0 * sb : 0.0)) + (d.metric2d ? goc::kMet * fb : 0.0);
    out[14] = d.nx;
    out[15] = d.ny;
    return GOC_OK;
}

int goc_lbm_derived(const goc_lbm_t* h, double out[16]) { return goc_lbm_derived_run(h, 0, out); }

int goc_lbm_metric(const goc_lbm_t* h, double* h1, double* th11, double* h2, double* th22)
{
    if (!h) return fail(GOC_EINVAL, "handle is NULL");
    if (h->m2d) return fail(GOC_EINVAL, "the run has a 2-D metric: use goc_lbm_metric_2d");
    const RunDesc& d = h->runs[0];
    if (h1) HIPOK(hipMemcpy(h1, h->h1_d + d.col_off, d.nx * 8, hipMemcpyDeviceToHost));
    if (th11) HIPOK(hipMemcpy(th11, h->th11_d + d.col_off, d.nx * 8, hipMemcpyDeviceToHost));
    if (h2) HIPOK(hipMemcpy(h2, h->h2_d + d.row_off, d.ny * 8, hipMemcpyDeviceToHost));
    if (th22) HIPOK(hipMemcpy(th22, h->th22_d + d.row_off, d.ny * 8, hipMemcpyDeviceToHost));
    return GOC_OK;
}

int goc_lbm_metric_2d(const goc_lbm_t* h, int32_t run, double* h1, double* h2, double* th11, double* th12,
                      double* th21, double* th22)
{
    if (!h) return fail(GOC_EINVAL, "handle is NULL");
    if (run < 0 || run >= h->nruns) return fail(GOC_EINVAL, "run %d outside [0, %d)", run, h->nruns);
    const RunDesc& d = h->runs[run];
    const int64_t N = (int64_t)d.nx * d.ny;
    double* outs[6] = {h1, h2, th11, th12, th21, th22};
    if (h->m2d) {
        const int planes[6] = {goc::M_H1, goc::M_H2, goc::M_TH11, goc::M_TH12, goc::M_TH21, goc::M_TH22};
        for (int k = 0; k < 6; ++k)
            if (outs[k])
                HIPOK(hipMemcpy(outs[k], h->met_d + d.met_off + planes[k] * N, N * 8, hipMemcpyDeviceToHost));
        return GOC_OK;
    }
    std::vector<double> c1(d.nx), t1(d.nx), c2(d.ny), t2(d.ny);
    HIPOK(hipMemcpy(c1.data(), h->h1_d + d.col_off, d.nx * 8, hipMemcpyDeviceToHost));
    HIPOK(hipMemcpy(t1.data(), h->th11_d + d.col_off, d.nx * 8, hipMemcpyDeviceToHost));
    HIPOK(hipMemcpy(c2.data(), h->h2_d + d.row_off, d.ny * 8, hipMemcpyDeviceToHost));
    HIPOK(hipMemcpy(t2.data(), h->th22_d + d.row_off, d.ny * 8, hipMemcpyDeviceToHost));
    for (int j = 0; j < d.ny; ++j)
        for (int i = 0; i < d.nx; ++i) {
            const int64_t n = (int64_t)j * d.nx + i;
            if (h1) h1[n] = c1[i];
            if (h2) h2[n] = c2[j];
            if (th11) th11[n] = t1[i];
            if (th12) th12[n] = 0.0;
            if (th21) th21[n] = 0.0;
            if (th22) th22[n] = t2[j];
        }
    return GOC_OK;
}

}  // extern "C"
