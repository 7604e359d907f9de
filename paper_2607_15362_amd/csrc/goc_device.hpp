// goc_device.hpp -- gfx950 device code of the GOC-LBM step: data layout,
// storage codecs and the per-node arithmetic.
//
// One fused pull-scheme kernel advances a whole time step of the
// central-moment MRT GOC-LBM (App. E of Yahia & Premnath, with the local
// shear stress of App. A and the boundary conditions of App. C) and, when
// enabled, the D2Q5 vector-distribution scheme of App. G.  A compile-time
// selector swaps the collision body for the raw-moment MRT model of the
// appendix that summarises it; the velocity-space SRT model of the
// appendix on velocity-space collisions is that model with every rate equal
// to 1/tau (f^eq = P^-1 m^eq and S = P^-1 sigma there, and P is linear).  The
// march takes a straight metric (h1(xi1), h2(xi2), theta12 = theta21 = 0;
// App. B(i)), which removes every theta12 / theta21 term and makes the
// effective force equal to its reduced form F~ (tau12 is not needed); general
// 2-D metrics take the curvilinear step of goc_curv.hpp, which keeps those
// terms (force_and_corrections_gen below).
//
// State layout in HBM (one plane per direction, rows interleaved): the
// element of plane a at node (i, j) is at a * plane + j * pitch + i, with
// plane the padded row length (nx rounded up to an odd number of 64-node
// pieces) and pitch the row stride, so that the planes of one row lie
// together: 9 population planes per row, or for an MHD run 20 (the nine
// population planes, one unused, then the ten D2Q5 planes from g_off =
// f_off + 10 plane, in the same pool); the two force planes have the row
// stride pitchF = 2 * plane.
//   slot(a, x) in plane a at the writer node x holds the population that
//   leaves x along e_a after collision, minus the rest-state population of
//   its reader (the node that pulls it), with the reader's wall condition
//   already applied by the writer (momentum-augmented bounce-back of App. C,
//   anti-bounce-back of App. G).  A reader y pulls slot(a, y - e_a) in the
//   interior and slot(opp(a), y) through a wall and gets its own deviation
//   d_a(y) = f_a(y) - f_a^rest(y) directly: streaming is a pure gather and
//   every slot has exactly one reader.  The rest state is the App. C initial
//   state at (rho0, U = 0); storing deviations keeps the full relative
//   precision of FP32 (and of the 16-bit forms) although the rest
//   populations themselves span h1 h2 (up to ~3) down to c_s^4/4 (~1e-8).
//   Lagged effective force: two planes per node (no streaming).
//
// Work decomposition: one wave64 work-group per (x-strip, y-segment).  The
// 64 lanes own 64 consecutive columns starting at a multiple of 64 (so that
// every row access of a wave is line-aligned); the wave marches up the rows
// of its segment keeping the moments of neighbouring rows in registers, so
// the finite differences of App. E step 3(a) need no second pass: the
// neighbouring columns come from neighbouring lanes, the two beyond the
// strip from lanes 0 and 63, which also pull and decode those halo nodes,
// and the halo rows from the march.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace goc {

constexpr int kQ = 9;
constexpr int kM = 5;
constexpr int kWave = 64;
constexpr int kOwn = kWave;   // columns owned per strip
constexpr int kTab = 8;   // doubles per column / row table entry
// Collision bodies selectable at compile time.
constexpr int kCollCentral = 0;
constexpr int kCollRaw = 1;

__host__ __device__ constexpr int ex_(int a) { return (a == 1 || a == 5 || a == 8) ? 1 : (a == 3 || a == 6 || a == 7) ? -1 : 0; }
__host__ __device__ constexpr int ey_(int a) { return (a == 2 || a == 5 || a == 6) ? 1 : (a == 4 || a == 7 || a == 8) ? -1 : 0; }
__host__ __device__ constexpr int opp_(int a) { return a == 0 ? 0 : (a <= 4 ? ((a + 1) % 4) + 1 : ((a - 5 + 2) % 4) + 5); }
// Scale class of a direction: 0 rest, 1 xi1-axis, 2 xi2-axis, 3 diagonal.
__host__ __device__ constexpr int cls_(int a) { return a == 0 ? 0 : (a == 1 || a == 3) ? 1 : (a == 2 || a == 4) ? 2 : 3; }

// Column / row metric tables (FP64, one entry of kTab doubles each):
//   col: h1, 1/h1, theta11, a1p, a1m, b1p, b1m, -
//   row: h2, 1/h2, theta22, a2p, a2m, b2p, b2m, -
// a1p = P0/2 (1/h1(i) - 1/h1(i+1)) is the difference between the rest-state
// xi1-axis population of a node and of its +xi1 neighbour divided by h2
// (zero when that neighbour lies beyond a wall); a1m the same toward -xi1;
// b1p, b1m the D2Q5 analogues W1 B0 (h1(i) - h1(i+-1)).  Rows likewise.
enum { T_H = 0, T_IH, T_TH, T_AP, T_AM, T_BP, T_BM };

// ---------------------------------------------------------------------------
// Run descriptor: one entry per independent run (a single run is a batch of 1).
// Indices of the ready-to-use step parameters of a run.
enum {
    P_CS2 = 0, P_ICS2, P_NU, P_ZETA, P_RHO0, P_P0, P_W, P_FX1 = P_W + 9, P_FX2, P_CSM2, P_ICSM2, P_TAUM,
    P_ITAUM, P_ETA, P_IMU, P_B0, P_WM0, P_WM1, P_SC, P_ISC = P_SC + 4, P_SCG = P_ISC + 4, P_ISCG, P_CWLO,
    P_CWHI, P_HWLO, P_HWHI, P_H1WLO, P_H1WHI, P_CXLO, P_CXHI, kNP
};

struct RunDesc {
    int32_t nx, ny, pitch;         // pitch: row stride of the slot pools (elements)
    int32_t bc_x, bc_y;            // 0 periodic, 1 wall
    int32_t strips, segs;          // launch geometry of this run
    int32_t first_block;           // first work-group of this run
    int32_t gi_terms, q3_sign, rho_terms, lid_corners, mhd;
    int32_t pitchF;                // row stride of the force pool
    int32_t metric2d;              // 1: general 2-D metric (per-node pool), else separable tables
    int64_t plane;                 // offset between planes within a row (the padded row length)
    int64_t f_off, F_off, g_off;   // element offsets of plane 0 in the f, force, g pools
    int64_t col_off, row_off;      // entry offsets into the column / row tables
    int64_t met_off, face_off;     // 2-D metric: offsets into the node pool and the face pool
    double cs2, nu, zeta;
    double omega[9];
    double Fx1, Fx2, rho0;
    double uw_lo, uw_hi;           // moving y-wall speeds (along xi1)
    double vw_lo, vw_hi;           // moving x-wall speeds (along xi2)
    double hw_lo, hw_hi;           // h2 on the y-wall faces
    double h1w_lo, h1w_hi;         // h1 on the x-wall faces
    double csm2, tau_m, eta, inv_mu, B0;
    double sc[4];                  // 16-bit storage: scale per direction class
    double scg;                    // 16-bit storage: scale of the D2Q5 deviations
    // the step's parameters ready to use (no arithmetic on the device), in
    // FP64 and rounded to FP32; filled by set_step_params
    double pd[kNP];
    float pf[kNP];
};

// Fill pd / pf from the fields above.
inline void set_step_params(RunDesc& d)
{
    double v[kNP];
    v[P_CS2] = d.cs2;
    v[P_ICS2] = 1.0 / d.cs2;
    v[P_NU] = d.nu;
    v[P_ZETA] = d.zeta;
    v[P_RHO0] = d.rho0;
    v[P_P0] = d.rho0 * d.cs2;
    for (int k = 0; k < 9; ++k) v[P_W + k] = d.omega[k];
    v[P_FX1] = d.Fx1;
    v[P_FX2] = d.Fx2;
    v[P_CSM2] = d.csm2;
    v[P_ICSM2] = d.csm2 > 0 ? 1.0 / d.csm2 : 0.0;
    v[P_TAUM] = d.tau_m;
    v[P_ITAUM] = 1.0 / d.tau_m;
    v[P_ETA] = d.eta;
    v[P_IMU] = d.inv_mu;
    v[P_B0] = d.B0;
    v[P_WM0] = 1.0 - 2.0 * d.csm2;
    v[P_WM1] = 0.5 * d.csm2;
    for (int k = 0; k < 4; ++k) {
        v[P_SC + k] = d.sc[k];
        v[P_ISC + k] = 1.0 / d.sc[k];
    }
    v[P_SCG] = d.scg;
    v[P_ISCG] = 1.0 / d.scg;
    v[P_CWLO] = d.hw_lo > 0 ? d.cs2 * d.uw_lo / (2.0 * d.hw_lo) : 0.0;
    v[P_CWHI] = d.hw_hi > 0 ? d.cs2 * d.uw_hi / (2.0 * d.hw_hi) : 0.0;
    v[P_HWLO] = d.hw_lo;
    v[P_HWHI] = d.hw_hi;
    v[P_H1WLO] = d.h1w_lo;
    v[P_H1WHI] = d.h1w_hi;
    v[P_CXLO] = d.h1w_lo > 0 ? d.cs2 * d.vw_lo / (2.0 * d.h1w_lo) : 0.0;
    v[P_CXHI] = d.h1w_hi > 0 ? d.cs2 * d.vw_hi / (2.0 * d.h1w_hi) : 0.0;
    for (int k = 0; k < kNP; ++k) {
        d.pd[k] = v[k];
        d.pf[k] = float(v[k]);
    }
}

template <class T> __device__ inline const T* step_params(const RunDesc& d);
template <> __device__ inline const double* step_params<double>(const RunDesc& d) { return d.pd; }
template <> __device__ inline const float* step_params<float>(const RunDesc& d) { return d.pf; }

// Pointers shared by all runs of a launch.
template <class S, class FT>
struct Pools {
    const S* fin;
    S* fout;
    const FT* Fin;
    FT* Fout;
    const S* gin;
    S* gout;
    const double* col;   // column tables
    const double* row;   // row tables
    const float* colf;   // the same tables rounded to FP32
    const float* rowf;
    // general 2-D metric: per-node planes (kMet of them, FP64 and FP32) and
    // the wall-face values (per row: h1 on the xi1 = 0 / nx faces; per
    // column: h2 on the xi2 = 0 / ny faces)
    const double* met;
    const float* metf;
    const double* face;
    // 16-bit storage: reference table of the slots (kRef floats per row of
    // each run; below).  A step decodes with ref_in and encodes with ref_out,
    // the same table except on the step that moves to a new one.
    const float* ref_in;
    const float* ref_out;
};

// Reference table of the 16-bit storage forms.  A 16-bit slot holds, scaled,
// the deviation of its population from the rest state minus the reference
// of its reader's row and direction: the mean over that row of the
// deviations pulled along that direction (entries 0-8; the D2Q5 slots of
// component c and direction a at 9 + 5 c + a), refreshed from the state
// every so many steps.  In a flow that varies little along a row (a channel,
// the developed Hartmann flow) the stored residual is then far smaller than
// the deviation itself, which carries the velocity, the lagged force and
// the magnetic field, and the format's rounding acts on the residual only.
constexpr int kRef = 20;    // floats per row (19 used)
constexpr int kRefG = 9;    // first D2Q5 entry

// Elements of one slot plane of a row: nx rounded up to whole pieces of 64
// nodes (one wave's columns), and an odd number of pieces, so that the
// planes of a row and the rows of a run do not all start a large power of
// two bytes apart (where they do, the many concurrent streams of a step
// crowd into a few of the memory channels: a 4096-column FP32 run with D2Q5
// slots stepped 142 us per launch with 65 pieces per plane against 152 us
// with 64).  The padding is never read or written.
// Planes of a slot-pool row before the D2Q5 planes of an MHD run (the nine
// population planes and one unused one); the ten D2Q5 planes follow, so an
// MHD row holds 2 kGPlanes planes.
constexpr int kGPlanes = 10;

__host__ __device__ constexpr int64_t padded_row(int nx)
{
    const int64_t p = (int64_t(nx) + 63) / 64;
    return 64 * (p % 2 ? p : p + 1);
}

// Planes of the 2-D metric pool, each nx * ny node values (row-major): the
// metric factors, their reciprocals, the curvature elements and the
// rest-state offsets of the four axis slots, f^rest_a(x) - f^rest_a(x + e_a)
// = (P0/2) (h2/h1 (x) - h2/h1 (x + e_a)) along xi1 and the xi2 analogue with
// h1/h2 (zero toward a wall, wrapped when periodic; computed in FP64, so the
// two offsets of one link are exact negatives also after rounding).
enum { M_H1 = 0, M_IH1, M_H2, M_IH2, M_TH11, M_TH12, M_TH21, M_TH22, M_AE, M_AW, M_AN, M_AS, kMet };

// ---------------------------------------------------------------------------
// Unbiased rounding of the stored values.  In a nearly steady flow a stored
// population changes by a fraction of its last place per step, so rounding
// to nearest repeats the same error on every step and the conserved moments
// drift linearly.  The writer therefore rounds base + increment
// stochastically: the rounding error is dithered by a uniform draw of one
// unit in the last place of the target format, which makes the expected
// stored value exact and the accumulated error a random walk.  The draws
// come from a counter-based hash of (node, population, step).

// 32-bit integer finaliser (the published "lowbias32" constants).
__host__ __device__ inline uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// a + b rounded stochastically to FP32.  The sum is formed in FP64, where it
// is exact (two FP32 values; b more than 29 binades below a is far below an
// FP32 ulp of the result anyway); adding 29 random bits below the FP32
// rounding point of the FP64 significand and truncating them lands on the
// upper neighbour (in magnitude, so for either sign) with probability equal
// to the discarded fraction: unbiased stochastic rounding.
__device__ inline float sr_add(float a, float b, uint32_t r)
{
    const double s = double(a) + double(b);
    const uint64_t u = (uint64_t(__double_as_longlong(s)) + (r >> 3)) & ~uint64_t(0x1FFFFFFF);
    return float(__longlong_as_double(int64_t(u)));
}

// ---------------------------------------------------------------------------
// Storage codecs: FP64 and FP32 store the deviation itself, the 16-bit forms
// store s * deviation with one scale s per direction class.  put / st_sr
// store base + inc with the unbiased rounding above (FP64: rounded to
// nearest) at an address / at an element index.
template <class S> struct Store;
template <> struct Store<double> {
    static constexpr bool scaled = false;
    __device__ static double dec(double v, double) { return v; }
    __device__ static double ld(const double* p, int64_t i, double) { return p[i]; }
    __device__ static void st(double* p, int64_t i, double v, double) { p[i] = v; }
    __device__ static double enc(double b, double inc, double, uint32_t) { return b + inc; }
    __device__ static void put(double* q, double b, double inc, double, uint32_t) { *q = b + inc; }
    __device__ static void st_sr(double* p, int64_t i, double b, double inc, double, uint32_t) { p[i] = b + inc; }
};
template <> struct Store<float> {
    static constexpr bool scaled = false;
    __device__ static float dec(float v, float) { return v; }
    __device__ static float ld(const float* p, int64_t i, float) { return p[i]; }
    __device__ static void st(float* p, int64_t i, float v, float) { p[i] = v; }
    __device__ static float enc(float b, float inc, float, uint32_t r) { return sr_add(b, inc, r); }
    __device__ static void put(float* q, float b, float inc, float, uint32_t r) { *q = sr_add(b, inc, r); }
    __device__ static void st_sr(float* p, int64_t i, float b, float inc, float, uint32_t r)
    {
        p[i] = sr_add(b, inc, r);
    }
};
// The 16-bit stores use the stochastic-rounding conversions of gfx950
// (v_cvt_sr_f16_f32 / v_cvt_sr_bf16_f32), which take the high 16 bits of
// the draw as the dither.
typedef __fp16 goc_f16x2 __attribute__((__vector_size__(2 * sizeof(__fp16))));
typedef __bf16 goc_bf16x2 __attribute__((__vector_size__(2 * sizeof(__bf16))));
template <> struct Store<__half> {
    static constexpr bool scaled = true;
    __device__ static float dec(__half v, float inv_s) { return __half2float(v) * inv_s; }
    __device__ static float ld(const __half* p, int64_t i, float inv_s) { return __half2float(p[i]) * inv_s; }
    __device__ static void st(__half* p, int64_t i, float v, float s) { p[i] = __float2half_rn(v * s); }
    __device__ static __half enc(float b, float inc, float s, uint32_t r)
    {
        // (the conversion writes the low half; the high half keeps the draw's
        // bits, which are dropped: no register needs clearing first)
        goc_f16x2 h = __builtin_bit_cast(goc_f16x2, r);
        h = __builtin_amdgcn_cvt_sr_f16_f32(h, (b + inc) * s, r, false);
        return __builtin_bit_cast(__half, uint16_t(__builtin_bit_cast(uint32_t, h)));
    }
    __device__ static void put(__half* q, float b, float inc, float s, uint32_t r) { *q = enc(b, inc, s, r); }
    __device__ static void st_sr(__half* p, int64_t i, float b, float inc, float s, uint32_t r)
    {
        put(p + i, b, inc, s, r);
    }
};
template <> struct Store<__hip_bfloat16> {
    static constexpr bool scaled = true;
    __device__ static float dec(__hip_bfloat16 v, float inv_s) { return __bfloat162float(v) * inv_s; }
    __device__ static float ld(const __hip_bfloat16* p, int64_t i, float inv_s) {
        return __bfloat162float(p[i]) * inv_s;
    }
    __device__ static void st(__hip_bfloat16* p, int64_t i, float v, float s) { p[i] = __float2bfloat16(v * s); }
    __device__ static __hip_bfloat16 enc(float b, float inc, float s, uint32_t r)
    {
        goc_bf16x2 h = __builtin_bit_cast(goc_bf16x2, r);   // (as for FP16)
        h = __builtin_amdgcn_cvt_sr_bf16_f32(h, (b + inc) * s, r, false);
        return __builtin_bit_cast(__hip_bfloat16, uint16_t(__builtin_bit_cast(uint32_t, h)));
    }
    __device__ static void put(__hip_bfloat16* q, float b, float inc, float s, uint32_t r)
    {
        *q = enc(b, inc, s, r);
    }
    __device__ static void st_sr(__hip_bfloat16* p, int64_t i, float b, float inc, float s, uint32_t r)
    {
        put(p + i, b, inc, s, r);
    }
};

// Reciprocal: correctly rounded division for FP64; for FP32 the hardware
// reciprocal refined by one fused Newton step r + r (1 - x r).
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// 1 / (a + b) for |a| >= |b|.  The rounding error of the FP32 sum is
// recovered exactly (Fast2Sum) and folded into the refined reciprocal, so a
// small deviation b keeps its full relative precision in the result.
__device__ inline double recip_sum(double a, double b) { return 1.0 / (a + b); }
__device__ inline float recip_sum(float a, float b)
{
    const float s = a + b;
    const float e = (a - s) + b;
    const float r = recip(s);
    return __builtin_fmaf(-r * e, r, r);
}

// Rest-state populations at (rho0, U = 0): P^-1 of the Sec. 3 equilibria.
__host__ __device__ inline double rest_pop(int a, double h1, double h2, double rho0, double cs2)
{
    const double P0 = rho0 * cs2, k22 = rho0 * cs2 * cs2;
    const int c = cls_(a);
    if (c == 0) return h1 * h2 * rho0 - (h2 / h1 + h1 / h2) * P0 + k22;
    if (c == 1) return 0.5 * (h2 / h1 * P0 - k22);
    if (c == 2) return 0.5 * (h1 / h2 * P0 - k22);
    return 0.25 * k22;
}

// ---------------------------------------------------------------------------
// Node-level arithmetic in deviation form.

template <class T>
struct NodeParams {
    T cs2, inv_cs2, nu, zeta, rho0, P0, w[9], Fx1, Fx2;
    int gi_terms, q3_sign, rho_terms;
    // MHD
    T csm2, inv_csm2, tau_m, inv_tau_m, eta, inv_mu, B0, W0, W1;
};

template <class T>
__device__ inline NodeParams<T> node_params(const RunDesc& d)
{
    const T* v = step_params<T>(d);
    NodeParams<T> p;
    p.cs2 = v[P_CS2];
    p.inv_cs2 = v[P_ICS2];
    p.nu = v[P_NU];
    p.zeta = v[P_ZETA];
    p.rho0 = v[P_RHO0];
    p.P0 = v[P_P0];
#pragma unroll
    for (int k = 0; k < 9; ++k) p.w[k] = v[P_W + k];
    p.Fx1 = v[P_FX1];
    p.Fx2 = v[P_FX2];
    p.gi_terms = d.gi_terms;
    p.q3_sign = d.q3_sign;
    p.rho_terms = d.rho_terms;
    p.csm2 = v[P_CSM2];
    p.inv_csm2 = v[P_ICSM2];
    p.tau_m = v[P_TAUM];
    p.inv_tau_m = v[P_ITAUM];
    p.eta = v[P_ETA];
    p.inv_mu = v[P_IMU];
    p.B0 = v[P_B0];
    p.W0 = v[P_WM0];
    p.W1 = v[P_WM1];
    return p;
}

// Opaque copies: an empty asm statement that takes the value as an
// in-out operand, so the compiler can no longer prove it loop-invariant.
// Applied to the lane constants at the top of each marched row, it keeps the
// loop from hoisting their many products out of the loop, where each would
// hold a vector register for the whole sweep.
__device__ inline void opaque_v(float& x) { asm volatile("" : "+v"(x)); }
__device__ inline void opaque_v(double& x) { asm volatile("" : "+v"(x)); }
__device__ inline void opaque_v(int32_t& x) { asm volatile("" : "+v"(x)); }
__device__ inline void opaque_v(uint32_t& x) { asm volatile("" : "+v"(x)); }

// Metric at one node.
template <class T>
struct NodeMetric {
    T h1, h2, ih1, ih2, th11, th22;
    T th12, th21;   // general 2-D metric only
};

// Effective force on a straight grid (Sec. 2.2 with theta12 = theta21 = 0):
//   F1 = h2 [F1ext - theta11 P + theta11 (tau11 - rho U1^2)],
//   F2 = h1 [F2ext - theta22 P + theta22 (tau22 - rho U2^2)],
// tau11, tau22 the normal viscous stresses of Sec. 2.2, and the equilibrium
// corrections n3^eq(1), n4^eq(1) of Sec. 4 on a straight grid.  The
// pressure P = P0 + c_s^2 (rho - rho0) is split so that its constant part
// is one product of constants and the varying part keeps the precision of
// the density deviation drho.
template <class T>
__device__ inline void force_and_corrections(const NodeParams<T>& p, const NodeMetric<T>& g, T rho, T drho,
                                             T U1, T U2, T d1U1, T d2U2, T d1r, T d2r, T Fe1, T Fe2,
                                             T& F1, T& F2, T& n3, T& n4)
{
    const T nu = p.nu, ze = p.zeta, ics = p.inv_cs2;
    const T h1 = g.h1, h2 = g.h2, ih1 = g.ih1, ih2 = g.ih2;
    const T dP = drho * p.cs2;
    const T a1 = d1U1 * ih1, a2 = d2U2 * ih2;
    const T tau11 = rho * ((ze + nu) * a1 + (ze - nu) * a2);
    const T tau22 = rho * ((ze + nu) * a2 + (ze - nu) * a1);
    F1 = h2 * (Fe1 + g.th11 * (tau11 - rho * U1 * U1 - dP)) - h2 * g.th11 * p.P0;
    F2 = h1 * (Fe2 + g.th22 * (tau22 - rho * U2 * U2 - dP)) - h1 * g.th22 * p.P0;

    const T r21 = h2 * ih1, r12 = h1 * ih2;          // h2/h1, h1/h2
    const T s1 = r21 * ih1, s2 = r12 * ih2;          // h2/h1^2, h1/h2^2
    const T u1s = U1 * U1 * ics, u2s = U2 * U2 * ics;
    T D31, D32, D33, D34, C3, D41, D42, D43, D44, C4;
    if (p.gi_terms) {
        D31 = rho * (ze * h2 * ics - (ze - nu) * ih2 - (T(2) * ze + nu + T(3) * ze * u1s) * s1);
        D32 = rho * (ze * h1 * ics - (ze - nu) * ih1 - (T(2) * ze + nu + T(3) * ze * u2s) * s2);
        D41 = rho * (nu * h2 * ics + (ze - nu) * ih2 - (ze + T(2) * nu + T(3) * nu * u1s) * s1);
        D42 = rho * (-nu * h1 * ics - (ze - nu) * ih1 + (ze + T(2) * nu + T(3) * nu * u2s) * s2);
        T b1, b2, c1, c2;
        if (p.rho_terms) {    // as printed
            b1 = ((T(3) - u1s) * s1 - h2 * ics - u2s * ih2) * U1;
            b2 = ((T(3) - u2s) * s2 - h1 * ics - u1s * ih1) * U2;
            c1 = ((T(3) - u1s) * s1 - h2 * ics + u2s * ih2) * U1;
            c2 = (-(T(3) - u2s) * s2 + h1 * ics - u1s * ih1) * U2;
        } else {              // from the Chapman-Enskog deviation terms
            b1 = ((T(3) + u1s) * s1 - h2 * ics) * U1;
            b2 = ((T(3) + u2s) * s2 - h1 * ics) * U2;
            c1 = b1;
            c2 = -b2;
        }
        D33 = -ze * b1;
        D34 = -ze * b2;
        D43 = -nu * c1;
        D44 = -nu * c2;
        const T g1 = U1 * (u1s + T(1)) * r21 * g.th11;
        const T g2 = U2 * (u2s + T(1)) * r12 * g.th22;
        C3 = T(2) * rho * ze * (g1 + g2);
        C4 = T(2) * rho * nu * (g1 - g2);
    } else {                  // App. B(ii)
        D31 = rho * (ze * h2 * ics - (ze - nu) * ih2 - (T(2) * ze + nu) * s1);
        D32 = rho * (ze * h1 * ics - (ze - nu) * ih1 - (T(2) * ze + nu) * s2);
        D41 = rho * (nu * h2 * ics + (ze - nu) * ih2 - (T(2) * nu + ze) * s1);
        D42 = rho * (-nu * h1 * ics - (ze - nu) * ih1 + (T(2) * nu + ze) * s2);
        D33 = D34 = D43 = D44 = T(0);
        const T g1 = U1 * r21 * g.th11, g2 = U2 * r12 * g.th22;
        C3 = T(2) * rho * ze * (g1 + g2);
        C4 = T(2) * rho * nu * (g1 - g2);
    }
    n3 = D31 * d1U1 + D32 * d2U2 + D33 * d1r + D34 * d2r + C3;
    n4 = D41 * d1U1 + D42 * d2U2 + D43 * d1r + D44 * d2r + C4;
}

// Effective force and equilibrium corrections on a general orthogonal grid
// (theta12, theta21 != 0): the normal stresses with their curvature parts
// tau^c (Sec. 2.2), the reduced force F~ (tau12 = 0), the local implicit
// shear stress from the non-equilibrium raw moment k'11 relaxed at omega5
// (App. A) and the full force F = F~ + 2 h theta tau12; the corrections
// n3^eq(1), n4^eq(1) of Sec. 4 with their tau^c and theta12 / theta21 terms
// (the App. B(ii) low-Mach set drops them, as on straight grids).  The
// pressure is split into P0 and c_s^2 (rho - rho0) as in the straight form.
template <class T>
__device__ inline void force_and_corrections_gen(const NodeParams<T>& p, const NodeMetric<T>& g, T rho, T drho,
                                                 T U1, T U2, T d1U1, T d2U2, T d1r, T d2r, T Fe1, T Fe2, T k11,
                                                 T& F1, T& F2, T& n3, T& n4)
{
    const T nu = p.nu, ze = p.zeta, ics = p.inv_cs2;
    const T h1 = g.h1, h2 = g.h2, ih1 = g.ih1, ih2 = g.ih2;
    const T t11 = g.th11, t12 = g.th12, t21 = g.th21, t22 = g.th22;
    const T dP = drho * p.cs2;
    const T a1 = d1U1 * ih1, a2 = d2U2 * ih2;
    const T tc11 = rho * ((ze + nu) * U2 * t12 + (ze - nu) * U1 * t21);
    const T tc22 = rho * ((ze + nu) * U1 * t21 + (ze - nu) * U2 * t12);
    const T tau11 = rho * ((ze + nu) * a1 + (ze - nu) * a2) + tc11;
    const T tau22 = rho * ((ze + nu) * a2 + (ze - nu) * a1) + tc22;
    const T uu = rho * U1 * U2;
    const T Ft1 = h2 * (Fe1 + (t21 - t11) * dP + t11 * (tau11 - rho * U1 * U1) - T(2) * t12 * uu
                        - t21 * (tau22 - rho * U2 * U2)) + h2 * (t21 - t11) * p.P0;
    const T Ft2 = h1 * (Fe2 + (t12 - t22) * dP + t22 * (tau22 - rho * U2 * U2) - T(2) * t21 * uu
                        - t12 * (tau11 - rho * U1 * U1)) + h1 * (t12 - t22) * p.P0;
    const T a = T(1) - T(0.5) * p.w[5];
    const T num = k11 + T(0.5) * (Ft1 * U2 * ih2 + Ft2 * U1 * ih1) - uu;
    const T tau12 = -a * num / (T(1) + a * (t12 * U2 + t21 * U1));
    F1 = Ft1 + T(2) * h2 * t12 * tau12;
    F2 = Ft2 + T(2) * h1 * t21 * tau12;

    const T r21 = h2 * ih1, r12 = h1 * ih2;
    const T s1 = r21 * ih1, s2 = r12 * ih2;
    const T u1s = U1 * U1 * ics, u2s = U2 * U2 * ics;
    T D31, D32, D33, D34, C3, D41, D42, D43, D44, C4;
    if (p.gi_terms) {
        D31 = rho * (ze * h2 * ics - (ze - nu) * ih2 - (T(2) * ze + nu + T(3) * ze * u1s) * s1);
        D32 = rho * (ze * h1 * ics - (ze - nu) * ih1 - (T(2) * ze + nu + T(3) * ze * u2s) * s2);
        D41 = rho * (nu * h2 * ics + (ze - nu) * ih2 - (ze + T(2) * nu + T(3) * nu * u1s) * s1);
        D42 = rho * (-nu * h1 * ics - (ze - nu) * ih1 + (ze + T(2) * nu + T(3) * nu * u2s) * s2);
        T b1, b2, c1, c2;
        if (p.rho_terms) {    // as printed
            b1 = ((T(3) - u1s) * s1 - h2 * ics - u2s * ih2) * U1;
            b2 = ((T(3) - u2s) * s2 - h1 * ics - u1s * ih1) * U2;
            c1 = ((T(3) - u1s) * s1 - h2 * ics + u2s * ih2) * U1;
            c2 = (-(T(3) - u2s) * s2 + h1 * ics - u1s * ih1) * U2;
        } else {              // from the Chapman-Enskog deviation terms
            b1 = ((T(3) + u1s) * s1 - h2 * ics) * U1;
            b2 = ((T(3) + u2s) * s2 - h1 * ics) * U2;
            c1 = b1;
            c2 = -b2;
        }
        D33 = -ze * b1;
        D34 = -ze * b2;
        D43 = -nu * c1;
        D44 = -nu * c2;
        const T g1 = U1 * (u1s + T(1)) * r21 * t11;
        const T g2 = U2 * (u2s + T(1)) * r12 * t22;
        const T hh = h1 * h2 * ics;
        const T q21 = U1 * (T(3) + u1s) * r21, q12 = U2 * (T(3) + u2s) * r12;
        C3 = T(2) * rho * ze * (g1 + g2) - (r21 * tc11 + r12 * tc22)
             - rho * ze * ((q21 + U1 * (T(2) * r12 - hh)) * t21 + (q12 + U2 * (T(2) * r21 - hh)) * t12);
        C4 = T(2) * rho * nu * (g1 - g2) - (r21 * tc11 - r12 * tc22)
             - rho * nu * ((q21 - U1 * (T(2) * r12 + hh)) * t21 + (-q12 + U2 * (T(2) * r21 + hh)) * t12);
    } else {                  // App. B(ii)
        D31 = rho * (ze * h2 * ics - (ze - nu) * ih2 - (T(2) * ze + nu) * s1);
        D32 = rho * (ze * h1 * ics - (ze - nu) * ih1 - (T(2) * ze + nu) * s2);
        D41 = rho * (nu * h2 * ics + (ze - nu) * ih2 - (T(2) * nu + ze) * s1);
        D42 = rho * (-nu * h1 * ics - (ze - nu) * ih1 + (T(2) * nu + ze) * s2);
        D33 = D34 = D43 = D44 = T(0);
        const T g1 = U1 * r21 * t11, g2 = U2 * r12 * t22;
        C3 = T(2) * rho * ze * (g1 + g2);
        C4 = T(2) * rho * nu * (g1 - g2);
    }
    n3 = D31 * d1U1 + D32 * d2U2 + D33 * d1r + D34 * d2r + C3;
    n4 = D41 * d1U1 + D42 * d2U2 + D43 * d1r + D44 * d2r + C4;
}

// Raw-moment deviations dm = P d (App. E step 1) for d = f - f^rest.
template <class T>
struct RawDev {
    T m00, m10, m01, m20, m02, m11, m21, m12, m22;
};

template <class T>
__device__ inline RawDev<T> raw_dev(const T* d)
{
    RawDev<T> m;
    const T s13 = d[1] + d[3], s24 = d[2] + d[4];
    const T a58 = d[5] + d[8], a67 = d[6] + d[7];
    const T p56 = d[5] + d[6], p78 = d[7] + d[8];
    m.m22 = p56 + p78;
    m.m00 = d[0] + s13 + s24 + m.m22;
    m.m10 = (d[1] - d[3]) + (a58 - a67);
    m.m01 = (d[2] - d[4]) + (p56 - p78);
    m.m20 = s13 + m.m22;
    m.m02 = s24 + m.m22;
    m.m11 = (d[5] - d[8]) - (d[6] - d[7]);
    m.m21 = p56 - p78;
    m.m12 = a58 - a67;
    return m;
}

// Population increments P^-1 n of raw-moment increments n (n00 = 0).
template <class T>
__device__ inline void pop_increments(T n10, T n01, T n20, T n02, T n11, T n21, T n12, T n22, T* inc)
{
    const T hx = T(0.5) * (n20 - n22), hy = T(0.5) * (n02 - n22);
    const T gx = T(0.5) * (n10 - n12), gy = T(0.5) * (n01 - n21);
    const T qa = T(0.25) * (n22 + n11), qb = T(0.25) * (n22 - n11);
    const T qc = T(0.25) * (n21 + n12), qd = T(0.25) * (n21 - n12);
    inc[0] = n22 - n20 - n02;
    inc[1] = hx + gx;
    inc[3] = hx - gx;
    inc[2] = hy + gy;
    inc[4] = hy - gy;
    inc[5] = qa + qc;
    inc[6] = qb + qd;
    inc[7] = qa - qc;
    inc[8] = qb - qd;
}

// Central-moment collision of App. E (steps 2-5) at one node, written as an
// increment: f~ = f + P^-1 F(U) dk, where dk = k~ - k are the changes of the
// central moments (relaxation plus sources; dk00 = 0) and F(U) maps central
// to raw moments.  Every step is linear in the moments, so this equals the
// transform chain of App. E; the rest-state moments (h1 h2 rho0, 0, 0,
// (h2/h1) P0, (h1/h2) P0, 0, 0, 0, rho0 c_s^4) cancel analytically and each
// population is rounded once, by the writer's final addition.  Forming the raw
// moments after collision as values of their own would round the slowly
// growing momentum on every step, a bias that FP32 accumulates.
// m: raw moments of the pre-collision deviations f - f^rest.
// Output: the population increments inc = f~ - f, added by the writer.
template <class T>
__device__ inline void cm_collide(const NodeParams<T>& p, const NodeMetric<T>& g, const RawDev<T>& m,
                                  T rho, T drho, T U1, T U2, T Fp1, T Fp2, T F1, T F2, T n3, T n4, T* inc)
{
    const T h1 = g.h1, h2 = g.h2;
    const T r21 = h2 * g.ih1, r12 = h1 * g.ih2;
    const T M0 = h1 * h2 * p.rho0, A = r21 * p.P0, Bm = r12 * p.P0;
    const T c00 = M0 + m.m00, c02 = Bm + m.m02;   // full moments
    // step 2: central moments (deviations from the rest central moments;
    // the first-order ones enter only through the identity below).  The
    // shift to central moments factors into a shift by U1 along xi1 and one
    // by U2 along xi2, each the binomial recurrence
    //   k0 = m0, k1 = m1 - U m0, k2 = m2 - U (m1 + k1);
    // the rest moments enter where they do not cancel (c00, c02 and, in the
    // second shift, A + a20).
    const T U11 = U1 * U1, U22 = U2 * U2, U12 = U1 * U2;
    const T a10 = m.m10 - U1 * c00, a20 = m.m20 - U1 * (m.m10 + a10);
    const T a11 = m.m11 - U1 * m.m01, a21 = m.m21 - U1 * (m.m11 + a11);
    const T a12 = m.m12 - U1 * c02, a22 = m.m22 - U1 * (m.m12 + a12);
    const T k01 = m.m01 - U2 * c00;
    const T k20 = a20;
    const T k02 = m.m02 - U2 * (m.m01 + k01);
    const T k11 = a11 - U2 * a10;
    const T k12 = a12 - U2 * (a11 + k11);
    const T k21 = a21 - U2 * (A + a20);
    const T k22 = a22 - U2 * (a21 + k21);
    // step 3: deviations of the central equilibria (binomial transform of the
    // Sec. 3 equilibria) with the corrections of Sec. 4
    const T h1m = h1 - T(1), h2m = h2 - T(1);
    const T q20 = r21 * h1m * h1m, q02 = r12 * h2m * h2m, q11 = h1m * h2m;
    T q21 = h1m * h1m * h2m * g.ih1, q12 = h1m * h2m * h2m * g.ih2;   // printed sign
    if (!p.q3_sign) { q21 = -q21; q12 = -q12; }                       // binomial transform
    const T rc = rho * p.cs2, drc = drho * p.cs2;
    const T e2s = q20 * rho * U11 + q02 * rho * U22 + (r21 + r12) * drc + n3;
    const T e2d = q20 * rho * U11 - q02 * rho * U22 + (r21 - r12) * drc + n4;
    const T e11 = q11 * rho * U12;
    const T e21 = q21 * rho * U11 * U2 - h2m * rc * U2 * g.ih1;
    const T e12 = q12 * rho * U1 * U22 - h1m * rc * U1 * g.ih2;
    const T e22 = drc * p.cs2;
    // central sources
    const T ih1m = g.ih1 - T(1), ih2m = g.ih2 - T(1);
    const T sa = T(2) * ih1m * F1 * U1, sb = T(2) * ih2m * F2 * U2;
    const T s11 = ih2m * F1 * U2 + ih1m * F2 * U1;
    // relaxation increments.  U carries the lagged force Fp, so the
    // first-order equilibria e10 = -(h1 - 1) h2 rho U1, e01 = -(h2 - 1) h1 rho U2
    // differ from k10, k01 by exactly Fp / 2: the identity is used instead of
    // the difference, which would turn a rounding bias of U into a momentum
    // source.
    const T* w = p.w;
    const T k2s = k20 + k02, k2d = k20 - k02;
    const T d10 = T(0.5) * w[1] * Fp1 + (T(1) - T(0.5) * w[1]) * F1;
    const T d01 = T(0.5) * w[2] * Fp2 + (T(1) - T(0.5) * w[2]) * F2;
    const T d2s = w[3] * (e2s - k2s) + (T(1) - T(0.5) * w[3]) * (sa + sb);
    const T d2d = w[4] * (e2d - k2d) + (T(1) - T(0.5) * w[4]) * (sa - sb);
    const T d11 = w[5] * (e11 - k11) + (T(1) - T(0.5) * w[5]) * s11;
    const T d21 = w[6] * (e21 - k21);
    const T d12 = w[7] * (e12 - k12);
    const T d22 = w[8] * (e22 - k22);
    const T d20 = T(0.5) * (d2s + d2d), d02 = T(0.5) * (d2s - d2d);
    // step 4: raw-moment increments, F(U) applied to dk (dk00 = 0): the
    // inverse shifts, by U2 along xi2 and then by U1 along xi1, each
    //   n0 = d0, n1 = d1 + U d0, n2 = d2 + U (d1 + n1)
    const T b11 = d11 + U2 * d10, b21 = d21 + U2 * d20;
    const T b02 = d02 + T(2) * U2 * d01;
    const T b12 = d12 + U2 * (d11 + b11), b22 = d22 + U2 * (d21 + b21);
    const T n10 = d10, n01 = d01;
    const T n20 = d20 + T(2) * U1 * d10;
    const T n02 = b02;
    const T n11 = b11 + U1 * d01;
    const T n21 = b21 + U1 * (b11 + n11);
    const T n12 = b12 + U1 * b02;
    const T n22 = b22 + U1 * (b12 + n12);
    // step 5: population increments P^-1 dn
    pop_increments(n10, n01, n20, n02, n11, n21, n12, n22, inc);
}

// Raw-moment MRT collision (the appendix summarising the raw-moment model),
// as an increment f~ = f + P^-1 dm with dm = m~ - m: the nine combined raw
// moments relax to the Sec. 3 equilibria (with the Sec. 4 corrections on
// k20 + k02 and k20 - k02) and gain the Sec. 3 sources.  Equilibria enter as
// deviations from the rest-state raw moments (h1 h2 rho0, 0, 0, (h2/h1) P0,
// (h1/h2) P0, 0, 0, 0, rho0 c_s^4), so no large value is formed; dk'00 = 0
// and the first-order increments use the lagged-force identity as in the
// central-moment body.  With every rate 1/tau this is the velocity-space
// SRT collision.
template <class T>
__device__ inline void raw_collide(const NodeParams<T>& p, const NodeMetric<T>& g, const RawDev<T>& m,
                                   T rho, T drho, T U1, T U2, T Fp1, T Fp2, T F1, T F2, T n3, T n4, T* inc)
{
    const T r21 = g.h2 * g.ih1, r12 = g.h1 * g.ih2;
    const T U11 = U1 * U1, U22 = U2 * U2;
    const T rc = rho * p.cs2, drc = drho * p.cs2;
    // equilibrium deviations
    const T e20 = r21 * (rho * U11 + drc), e02 = r12 * (rho * U22 + drc);
    const T e2s = e20 + e02 + n3, e2d = e20 - e02 + n4;
    const T e11 = rho * U1 * U2;
    const T e21 = (rc + rho * U11) * U2 * g.ih1;
    const T e12 = (rc + rho * U22) * U1 * g.ih2;
    const T e22 = drc * p.cs2 + rho * (p.cs2 * (U11 + U22) + U11 * U22);
    // sources
    const T sa = T(2) * F1 * U1 * g.ih1, sb = T(2) * F2 * U2 * g.ih2;
    const T s11 = F1 * U2 * g.ih2 + F2 * U1 * g.ih1;
    // relaxation increments
    const T* w = p.w;
    const T k2s = m.m20 + m.m02, k2d = m.m20 - m.m02;
    const T d10 = T(0.5) * w[1] * Fp1 + (T(1) - T(0.5) * w[1]) * F1;
    const T d01 = T(0.5) * w[2] * Fp2 + (T(1) - T(0.5) * w[2]) * F2;
    const T d2s = w[3] * (e2s - k2s) + (T(1) - T(0.5) * w[3]) * (sa + sb);
    const T d2d = w[4] * (e2d - k2d) + (T(1) - T(0.5) * w[4]) * (sa - sb);
    const T d11 = w[5] * (e11 - m.m11) + (T(1) - T(0.5) * w[5]) * s11;
    const T d21 = w[6] * (e21 - m.m21);
    const T d12 = w[7] * (e12 - m.m12);
    const T d22 = w[8] * (e22 - m.m22);
    const T d20 = T(0.5) * (d2s + d2d), d02 = T(0.5) * (d2s - d2d);
    pop_increments(d10, d01, d20, d02, d11, d21, d12, d22, inc);
}

// D2Q5 induction scheme of App. G on a straight grid (Y = 0: no source), in
// deviation form: dg[c][a] = g_ca - W_a h1 h2 B_rest,c with B_rest = (0, B0).
// Computes B, the local derivatives dB from the non-equilibrium first
// moments, J3, the Lorentz force and (if dgi != nullptr) the collision
// increments g~ - g.
template <class T>
__device__ inline void mie_node(const NodeParams<T>& p, const NodeMetric<T>& g, const T (*dg)[kM],
                                T U1, T U2, T& B1, T& B2, T& FL1, T& FL2, T (*dgi)[kM])
{
    const T h1 = g.h1, h2 = g.h2, hh = h1 * h2, ihh = g.ih1 * g.ih2;
    T S[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) S[i] = dg[i][0] + dg[i][1] + dg[i][2] + dg[i][3] + dg[i][4];
    B1 = S[0] * ihh;
    B2 = p.B0 + S[1] * ihh;
    const T B[2] = {B1, B2};
    // flux tensor A_i1 = U1 B_i - B1 U_i, A_i2 = U2 B_i - B2 U_i
    const T A12 = U2 * B1 - B2 * U1;
    const T A21 = U1 * B2 - B1 * U2;
    const T L1eq[2] = {T(0), h2 * A21};   // first moments of g^eq(0) along xi1 (A11 = 0)
    const T L2eq[2] = {h1 * A12, T(0)};   // along xi2 (A22 = 0)
    const T cs = p.csm2, tm = p.tau_m;
    const T den1 = recip(cs * (T(0.5) * hh + (tm - T(0.5)) * h2 * g.ih1));
    const T den2 = recip(cs * (T(0.5) * hh + (tm - T(0.5)) * h1 * g.ih2));
    T dB1[2], dB2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const T L1 = (dg[i][1] - dg[i][3]) - L1eq[i];
        const T L2 = (dg[i][2] - dg[i][4]) - L2eq[i];
        dB1[i] = -(L1 + T(0.5) * cs * h1 * hh * g.th11 * B[i]) * den1;
        dB2[i] = -(L2 + T(0.5) * cs * hh * h2 * g.th22 * B[i]) * den2;
    }
    const T J3 = p.inv_mu * ihh * (h2 * dB1[1] - h1 * dB2[0]);
    FL1 = -J3 * B2;
    FL2 = J3 * B1;
    if (dgi == nullptr) return;
    const T itm = p.inv_tau_m, ics = p.inv_csm2;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const T Lc1 = p.eta * ((hh - h2 * g.ih1) * dB1[i] + h1 * hh * g.th11 * B[i]);
        const T Lc2 = p.eta * ((hh - h1 * g.ih2) * dB2[i] + hh * h2 * g.th22 * B[i]);
        const T m1 = (L1eq[i] + Lc1) * ics, m2 = (L2eq[i] + Lc2) * ics;
        const T base = S[i];   // h1 h2 (B_i - B_rest,i)
        const T e1 = p.W1 * (base + m1), e3 = p.W1 * (base - m1);
        const T e2 = p.W1 * (base + m2), e4 = p.W1 * (base - m2);
        dgi[i][1] = (e1 - dg[i][1]) * itm;
        dgi[i][2] = (e2 - dg[i][2]) * itm;
        dgi[i][3] = (e3 - dg[i][3]) * itm;
        dgi[i][4] = (e4 - dg[i][4]) * itm;
        // sum of g^eq = sum of g = h1 h2 B_i: the rest population takes
        // minus the other increments, so that B is conserved to the rounding
        // of the increments rather than that of the (larger) equilibria,
        // whose error would repeat on every step of a steady flow
        dgi[i][0] = -((dgi[i][1] + dgi[i][3]) + (dgi[i][2] + dgi[i][4]));
    }
}

// ---------------------------------------------------------------------------
// Geometry helpers of the strip / segment decomposition.

// Balanced split of ny rows into segs segments of at least two rows.
// Rows [y0, y1) of segment s of segs: whole groups of kRowGroup rows (the
// step kernel marches a group per loop pass); the last segment also takes
// the ny mod kRowGroup rows left over, so that every segment of a run with
// ny >= kRowGroup has at least kRowGroup rows (the one-sided difference at
// the top wall then finds row ny - 3 in the march).  segs <= row_groups(ny).
constexpr int kRowGroup = 4;
__host__ __device__ inline int row_groups(int ny) { return ny / kRowGroup > 1 ? ny / kRowGroup : 1; }
__host__ __device__ inline void seg_rows(int ny, int segs, int s, int& y0, int& y1)
{
    const int64_t groups = row_groups(ny);
    y0 = kRowGroup * (int)((groups * s) / segs);
    y1 = s == segs - 1 ? ny : kRowGroup * (int)((groups * (s + 1)) / segs);
}

// First column covered by lane 0 of strip k.  With x-walls the last strip
// is shifted so that it always holds the three columns the one-sided
// difference at the last column needs.
__host__ __device__ inline int lane_base(int nx, int bc_x, int k)
{
    const int x0 = k * kOwn;
    // with x-walls a last strip holding only the wall column starts one
    // column early: the one-sided difference there needs the two columns
    // before it, which lane 0 and lane 0's halo then provide
    if (bc_x && nx - x0 == 1) return x0 - 1;
    return x0;
}

template <class T>
__device__ inline T shfl(T v, int src) { return __shfl(v, src, kWave); }

}  // namespace goc
