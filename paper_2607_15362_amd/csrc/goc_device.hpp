// goc_device.hpp -- gfx950 device code of the GOC-LBM step.
//
// One fused pull-scheme kernel advances a whole time step of the
// central-moment MRT GOC-LBM (App. E of Yahia & Premnath, with the local
// shear stress of App. A and the boundary conditions of App. C) and, when
// enabled, the D2Q5 vector-distribution scheme of App. G.  The metric is
// straight (h1(xi1), h2(xi2), theta12 = theta21 = 0; App. B(i)), which
// removes every theta12 / theta21 term and makes the effective force equal
// to its reduced form F~ (tau12 is not needed).
//
// State layout in HBM (structure of arrays, one plane per direction):
//   slot(a, x) in plane a at the writer node x holds the post-collision
//   population that leaves x along e_a, with the wall condition of its
//   reader already applied by the writer (momentum-augmented bounce-back
//   of App. C, anti-bounce-back of App. G).  A reader y therefore pulls
//   f_a(y) = slot(a, y - e_a) in the interior and slot(opp(a), y) through a
//   wall: streaming is a pure gather and every slot has exactly one reader.
//   Lagged effective force: two planes per node (no streaming).
//
// Work decomposition: one wave64 work-group per (x-strip, y-segment).  The
// 64 lanes cover 64 consecutive columns, of which the inner 62 are owned;
// the wave marches up the rows of its segment keeping the moments of rows
// j-2 .. j+1 in registers, so the finite differences of App. E step 3(a)
// need no second pass: halo columns come from neighbouring lanes, halo
// rows from the march (recomputed at segment ends from the pulled
// populations).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace goc {

constexpr int kQ = 9;
constexpr int kM = 5;
constexpr int kWave = 64;
constexpr int kOwn = kWave - 2;

__host__ __device__ constexpr int ex_(int a) { return (a == 1 || a == 5 || a == 8) ? 1 : (a == 3 || a == 6 || a == 7) ? -1 : 0; }
__host__ __device__ constexpr int ey_(int a) { return (a == 2 || a == 5 || a == 6) ? 1 : (a == 4 || a == 7 || a == 8) ? -1 : 0; }
__host__ __device__ constexpr int opp_(int a) { return a == 0 ? 0 : (a <= 4 ? ((a + 1) % 4) + 1 : ((a - 5 + 2) % 4) + 5); }

// ---------------------------------------------------------------------------
// Run descriptor: one entry per independent run (a single run is a batch of 1).
struct RunDesc {
    int32_t nx, ny, pitch;
    int32_t bc_x, bc_y;            // 0 periodic, 1 wall
    int32_t strips, segs;          // launch geometry of this run
    int32_t first_block;           // first work-group of this run
    int32_t gi_terms, q3_sign, rho_terms, lid_corners, mhd;
    int32_t pad_;
    int64_t plane;                 // elements per plane (row pitch * ny + padding)
    int64_t f_off, F_off, g_off;   // element offsets of plane 0 in the f, force, g pools
    int64_t metric_off_x, metric_off_y;   // offsets into the metric pools
    double cs2, nu, zeta;
    double omega[9];
    double Fx1, Fx2, rho0;
    double uw_lo, uw_hi;           // moving y-wall speeds
    double hw_lo, hw_hi;           // h2 on the y-wall faces
    double h1w_lo, h1w_hi;         // h1 on the x-wall faces
    double csm2, tau_m, eta, inv_mu, B0;
    double sc[4];                  // 16-bit storage: scale per direction class
    double scg;                    // 16-bit storage: scale of the D2Q5 deviations
};

// Pointers shared by all runs of a launch.
template <class S, class FT>
struct Pools {
    const S* fin;
    S* fout;
    const FT* Fin;
    FT* Fout;
    const S* gin;
    S* gout;
    const double* h1;    // [sum nx]
    const double* th11;
    const double* h2;    // [sum ny]
    const double* th22;
};

// ---------------------------------------------------------------------------
// Storage codecs.  FP64 / FP32 store populations as they are.  The 16-bit
// forms store s * (value - rest), rest being the writer node's population at
// rest (rho0, U = 0, App. C closed form), with one scale s per direction class.
template <class S> struct Store;
template <> struct Store<double> {
    static constexpr bool dev = false;
    __device__ static double ld(const double* p, int64_t i, double, double) { return p[i]; }
    __device__ static void st(double* p, int64_t i, double v, double, double) { p[i] = v; }
};
template <> struct Store<float> {
    static constexpr bool dev = false;
    __device__ static float ld(const float* p, int64_t i, float, float) { return p[i]; }
    __device__ static void st(float* p, int64_t i, float v, float, float) { p[i] = v; }
};
template <> struct Store<__half> {
    static constexpr bool dev = true;
    __device__ static float ld(const __half* p, int64_t i, float rest, float inv_s) {
        return fmaf(__half2float(p[i]), inv_s, rest);
    }
    __device__ static void st(__half* p, int64_t i, float v, float rest, float s) {
        p[i] = __float2half_rn((v - rest) * s);
    }
};
template <> struct Store<__hip_bfloat16> {
    static constexpr bool dev = true;
    __device__ static float ld(const __hip_bfloat16* p, int64_t i, float rest, float inv_s) {
        return fmaf(__bfloat162float(p[i]), inv_s, rest);
    }
    __device__ static void st(__hip_bfloat16* p, int64_t i, float v, float rest, float s) {
        p[i] = __float2bfloat16((v - rest) * s);
    }
};

// Scale class of a direction: 0 rest, 1 xi1-axis, 2 xi2-axis, 3 diagonal.
__host__ __device__ constexpr int cls_(int a) { return a == 0 ? 0 : (a == 1 || a == 3) ? 1 : (a == 2 || a == 4) ? 2 : 3; }

// Rest-state populations at (rho0, U = 0): P^-1 of the Sec. 3 equilibria.
template <class T>
__device__ inline T rest_pop(int a, T h1, T h2, T rho0, T cs2) {
    const T P0 = rho0 * cs2, k22 = rho0 * cs2 * cs2;
    const int c = cls_(a);
    if (c == 0) return h1 * h2 * rho0 - (h2 / h1 + h1 / h2) * P0 + k22;
    if (c == 1) return T(0.5) * (h2 / h1 * P0 - k22);
    if (c == 2) return T(0.5) * (h1 / h2 * P0 - k22);
    return T(0.25) * k22;
}

// ---------------------------------------------------------------------------
// Node-level arithmetic.

template <class T>
struct NodeParams {
    T cs2, inv_cs2, nu, zeta, w[9], Fx1, Fx2;
    int gi_terms, q3_sign, rho_terms;
    // MHD
    T csm2, inv_csm2, tau_m, inv_tau_m, eta, inv_mu, B0, W0, W1;
};

// Effective force on a straight grid (Sec. 2.2 with theta12 = theta21 = 0):
//   F1 = h2 [F1ext - theta11 P + theta11 (tau11 - rho U1^2)],
//   F2 = h1 [F2ext - theta22 P + theta22 (tau22 - rho U2^2)],
// tau11, tau22 the normal viscous stresses of Sec. 2.2.
// Equilibrium corrections n3^eq(1), n4^eq(1) of Sec. 5 on a straight grid.
template <class T>
__device__ inline void force_and_corrections(const NodeParams<T>& p, T h1, T h2, T th11, T th22,
                                             T rho, T U1, T U2, T d1U1, T d2U2, T d1r, T d2r,
                                             T Fe1, T Fe2, T& F1, T& F2, T& n3, T& n4)
{
    const T nu = p.nu, ze = p.zeta, ics = p.inv_cs2;
    const T ih1 = T(1) / h1, ih2 = T(1) / h2;
    const T P = rho * p.cs2;
    const T a1 = d1U1 * ih1, a2 = d2U2 * ih2;
    const T tau11 = rho * ((ze + nu) * a1 + (ze - nu) * a2);
    const T tau22 = rho * ((ze + nu) * a2 + (ze - nu) * a1);
    F1 = h2 * (Fe1 - th11 * P + th11 * (tau11 - rho * U1 * U1));
    F2 = h1 * (Fe2 - th22 * P + th22 * (tau22 - rho * U2 * U2));

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
        const T g1 = U1 * (u1s + T(1)) * r21 * th11;
        const T g2 = U2 * (u2s + T(1)) * r12 * th22;
        C3 = T(2) * rho * ze * (g1 + g2);
        C4 = T(2) * rho * nu * (g1 - g2);
    } else {                  // App. B(ii)
        D31 = rho * (ze * h2 * ics - (ze - nu) * ih2 - (T(2) * ze + nu) * s1);
        D32 = rho * (ze * h1 * ics - (ze - nu) * ih1 - (T(2) * ze + nu) * s2);
        D41 = rho * (nu * h2 * ics + (ze - nu) * ih2 - (T(2) * nu + ze) * s1);
        D42 = rho * (-nu * h1 * ics - (ze - nu) * ih1 + (T(2) * nu + ze) * s2);
        D33 = D34 = D43 = D44 = T(0);
        const T g1 = U1 * r21 * th11, g2 = U2 * r12 * th22;
        C3 = T(2) * rho * ze * (g1 + g2);
        C4 = T(2) * rho * nu * (g1 - g2);
    }
    n3 = D31 * d1U1 + D32 * d2U2 + D33 * d1r + D34 * d2r + C3;
    n4 = D41 * d1U1 + D42 * d2U2 + D43 * d1r + D44 * d2r + C4;
}

// Central-moment collision of App. E (steps 1-5) at one node.
// In: pre-collision populations f, fields rho, U, effective force F,
// corrections n3, n4.  Out: post-collision populations ft.
template <class T>
__device__ inline void cm_collide(const NodeParams<T>& p, T h1, T h2, const T* f, T rho, T U1,
                                  T U2, T F1, T F2, T n3, T n4, T* ft)
{
    // step 1: raw moments (bare basis k00 k10 k01 k20 k02 k11 k21 k12 k22)
    const T s13 = f[1] + f[3], s24 = f[2] + f[4];
    const T d13 = f[1] - f[3], d24 = f[2] - f[4];
    const T a58 = f[5] + f[8], a67 = f[6] + f[7];    // e2-odd pairs summed in e1
    const T p56 = f[5] + f[6], p78 = f[7] + f[8];
    const T q58 = f[5] - f[8], q67 = f[6] - f[7];
    const T sd = p56 + p78;                           // k22
    const T m00 = f[0] + s13 + s24 + sd;
    const T m10 = d13 + (a58 - a67);
    const T m01 = d24 + (p56 - p78);
    const T m20 = s13 + sd;
    const T m02 = s24 + sd;
    const T m11 = q58 - q67;
    const T m21 = p56 - p78;
    const T m12 = a58 - a67;
    const T m22 = sd;
    // step 2: central moments with U
    const T U11 = U1 * U1, U22 = U2 * U2, U12 = U1 * U2;
    const T k10 = m10 - U1 * m00;
    const T k01 = m01 - U2 * m00;
    const T k20 = m20 - T(2) * U1 * m10 + U11 * m00;
    const T k02 = m02 - T(2) * U2 * m01 + U22 * m00;
    const T k11 = m11 - U2 * m10 - U1 * m01 + U12 * m00;
    const T k21 = m21 - T(2) * U1 * m11 + U11 * m01 - U2 * m20 + T(2) * U12 * m10 - U11 * U2 * m00;
    const T k12 = m12 - T(2) * U2 * m11 + U22 * m10 - U1 * m02 + T(2) * U12 * m01 - U1 * U22 * m00;
    const T k22 = m22 - T(2) * U1 * m12 + U11 * m02 - T(2) * U2 * m21 + T(4) * U12 * m11
                - T(2) * U11 * U2 * m01 + U22 * m20 - T(2) * U1 * U22 * m10 + U11 * U22 * m00;
    // step 3: central equilibria (binomial transform of the Sec. 3 equilibria) + corrections
    const T h1m = h1 - T(1), h2m = h2 - T(1);
    const T r21 = h2 / h1, r12 = h1 / h2;
    const T q20 = r21 * h1m * h1m, q02 = r12 * h2m * h2m, q11 = h1m * h2m;
    T q21 = h1m * h1m * h2m / h1, q12 = h1m * h2m * h2m / h2;   // printed sign
    if (!p.q3_sign) { q21 = -q21; q12 = -q12; }                 // binomial transform
    const T rc = rho * p.cs2;
    const T e10 = -h1m * h2 * rho * U1;
    const T e01 = -h2m * h1 * rho * U2;
    const T e2s = q20 * rho * U11 + q02 * rho * U22 + (r21 + r12) * rc + n3;
    const T e2d = q20 * rho * U11 - q02 * rho * U22 + (r21 - r12) * rc + n4;
    const T e11 = q11 * rho * U12;
    const T e21 = q21 * rho * U11 * U2 - h2m * rc * U2 / h1;
    const T e12 = q12 * rho * U1 * U22 - h1m * rc * U1 / h2;
    const T e22 = rc * p.cs2;
    // central sources
    const T ih1m = T(1) / h1 - T(1), ih2m = T(1) / h2 - T(1);
    const T sa = T(2) * ih1m * F1 * U1, sb = T(2) * ih2m * F2 * U2;
    const T s2s = sa + sb, s2d = sa - sb;
    const T s11 = ih2m * F1 * U2 + ih1m * F2 * U1;
    // relaxation (k00 kept exactly, mass conserved to rounding)
    const T* w = p.w;
    const T k2s = k20 + k02, k2d = k20 - k02;
    const T t10 = k10 + w[1] * (e10 - k10) + (T(1) - T(0.5) * w[1]) * F1;
    const T t01 = k01 + w[2] * (e01 - k01) + (T(1) - T(0.5) * w[2]) * F2;
    const T t2s = k2s + w[3] * (e2s - k2s) + (T(1) - T(0.5) * w[3]) * s2s;
    const T t2d = k2d + w[4] * (e2d - k2d) + (T(1) - T(0.5) * w[4]) * s2d;
    const T t11 = k11 + w[5] * (e11 - k11) + (T(1) - T(0.5) * w[5]) * s11;
    const T t21 = k21 + w[6] * (e21 - k21);
    const T t12 = k12 + w[7] * (e12 - k12);
    const T t22 = k22 + w[8] * (e22 - k22);
    const T t20 = T(0.5) * (t2s + t2d), t02 = T(0.5) * (t2s - t2d);
    const T t00 = m00;
    // step 4: raw moments from central ones, F(-U)
    const T n10 = t10 + U1 * t00;
    const T n01 = t01 + U2 * t00;
    const T n20 = t20 + T(2) * U1 * t10 + U11 * t00;
    const T n02 = t02 + T(2) * U2 * t01 + U22 * t00;
    const T n11 = t11 + U2 * t10 + U1 * t01 + U12 * t00;
    const T n21 = t21 + T(2) * U1 * t11 + U11 * t01 + U2 * t20 + T(2) * U12 * t10 + U11 * U2 * t00;
    const T n12 = t12 + T(2) * U2 * t11 + U22 * t10 + U1 * t02 + T(2) * U12 * t01 + U1 * U22 * t00;
    const T n22 = t22 + T(2) * U1 * t12 + U11 * t02 + T(2) * U2 * t21 + T(4) * U12 * t11
                + T(2) * U11 * U2 * t01 + U22 * t20 + T(2) * U1 * U22 * t10 + U11 * U22 * t00;
    // step 5: populations, P^-1
    ft[0] = t00 - n20 - n02 + n22;
    const T hx = T(0.5) * (n20 - n22), hy = T(0.5) * (n02 - n22);
    const T gx = T(0.5) * (n10 - n12), gy = T(0.5) * (n01 - n21);
    ft[1] = hx + gx;
    ft[3] = hx - gx;
    ft[2] = hy + gy;
    ft[4] = hy - gy;
    const T qa = T(0.25) * (n22 + n11), qb = T(0.25) * (n22 - n11);
    const T qc = T(0.25) * (n21 + n12), qd = T(0.25) * (n21 - n12);
    ft[5] = qa + qc;
    ft[6] = qb + qd;
    ft[7] = qa - qc;
    ft[8] = qb - qd;
}

// D2Q5 induction scheme of App. G on a straight grid (Y = 0: no source).
// gb[c][a]: transformed populations of component c.  Computes B, the local
// derivatives dB from the non-equilibrium first moments, J3, the Lorentz
// force, and (if gt != nullptr) the post-collision populations.
template <class T>
__device__ inline void mie_node(const NodeParams<T>& p, T h1, T h2, T th11, T th22,
                                const T (*gb)[kM], T U1, T U2, T& B1, T& B2, T& FL1, T& FL2,
                                T (*gt)[kM])
{
    const T hh = h1 * h2, ihh = T(1) / hh;
    B1 = (gb[0][0] + gb[0][1] + gb[0][2] + gb[0][3] + gb[0][4]) * ihh;
    B2 = (gb[1][0] + gb[1][1] + gb[1][2] + gb[1][3] + gb[1][4]) * ihh;
    const T B[2] = {B1, B2};
    // flux tensor A_i1 = U1 B_i - B1 U_i, A_i2 = U2 B_i - B2 U_i
    const T A11 = T(0), A12 = U2 * B1 - B2 * U1;
    const T A21 = U1 * B2 - B1 * U2, A22 = T(0);
    const T L1eq[2] = {h2 * A11, h2 * A21};   // first moments of g^eq(0) along xi1
    const T L2eq[2] = {h1 * A12, h1 * A22};   // along xi2
    const T cs = p.csm2, tm = p.tau_m;
    const T den1 = T(1) / (cs * (T(0.5) * hh + (tm - T(0.5)) * h2 / h1));
    const T den2 = T(1) / (cs * (T(0.5) * hh + (tm - T(0.5)) * h1 / h2));
    T dB1[2], dB2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const T L1 = (gb[i][1] - gb[i][3]) - L1eq[i];
        const T L2 = (gb[i][2] - gb[i][4]) - L2eq[i];
        dB1[i] = -(L1 + T(0.5) * cs * h1 * hh * th11 * B[i]) * den1;
        dB2[i] = -(L2 + T(0.5) * cs * hh * h2 * th22 * B[i]) * den2;
    }
    const T J3 = p.inv_mu * ihh * (h2 * dB1[1] - h1 * dB2[0]);
    FL1 = -J3 * B2;
    FL2 = J3 * B1;
    if (gt == nullptr) return;
    const T itm = p.inv_tau_m, ics = p.inv_csm2;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const T Lc1 = p.eta * ((hh - h2 / h1) * dB1[i] + h1 * hh * th11 * B[i]);
        const T Lc2 = p.eta * ((hh - h1 / h2) * dB2[i] + hh * h2 * th22 * B[i]);
        const T m1 = (L1eq[i] + Lc1) * ics, m2 = (L2eq[i] + Lc2) * ics;
        const T base = hh * B[i];
        const T geq0 = p.W0 * base;
        const T geq1 = p.W1 * (base + m1), geq3 = p.W1 * (base - m1);
        const T geq2 = p.W1 * (base + m2), geq4 = p.W1 * (base - m2);
        gt[i][0] = gb[i][0] - (gb[i][0] - geq0) * itm;
        gt[i][1] = gb[i][1] - (gb[i][1] - geq1) * itm;
        gt[i][2] = gb[i][2] - (gb[i][2] - geq2) * itm;
        gt[i][3] = gb[i][3] - (gb[i][3] - geq3) * itm;
        gt[i][4] = gb[i][4] - (gb[i][4] - geq4) * itm;
    }
}

template <class T>
__device__ inline NodeParams<T> node_params(const RunDesc& d)
{
    NodeParams<T> p;
    p.cs2 = T(d.cs2);
    p.inv_cs2 = T(1.0 / d.cs2);
    p.nu = T(d.nu);
    p.zeta = T(d.zeta);
#pragma unroll
    for (int k = 0; k < 9; ++k) p.w[k] = T(d.omega[k]);
    p.Fx1 = T(d.Fx1);
    p.Fx2 = T(d.Fx2);
    p.gi_terms = d.gi_terms;
    p.q3_sign = d.q3_sign;
    p.rho_terms = d.rho_terms;
    p.csm2 = T(d.csm2);
    p.inv_csm2 = T(1.0 / d.csm2);
    p.tau_m = T(d.tau_m);
    p.inv_tau_m = T(1.0 / d.tau_m);
    p.eta = T(d.eta);
    p.inv_mu = T(d.inv_mu);
    p.B0 = T(d.B0);
    p.W0 = T(1.0 - 2.0 * d.csm2);
    p.W1 = T(0.5 * d.csm2);
    return p;
}

// ---------------------------------------------------------------------------
// Geometry helpers of the strip / segment decomposition.

// Balanced split of ny rows into segs segments of at least two rows.
__device__ inline void seg_rows(int ny, int segs, int s, int& y0, int& y1)
{
    y0 = (int)(((int64_t)ny * s) / segs);
    y1 = (int)(((int64_t)ny * (s + 1)) / segs);
}

// First column covered by lane 0 of strip k.  With x-walls the last strip
// is shifted so that it always holds the three columns the one-sided
// difference at the last column needs.
__device__ inline int lane_base(int nx, int bc_x, int k)
{
    const int x0 = k * kOwn;
    if (bc_x && nx - x0 < 2 && nx >= kWave - 1) return nx - (kWave - 1);
    return x0 - 1;
}

template <class T>
__device__ inline T shfl(T v, int src) { return __shfl(v, src, kWave); }

}  // namespace goc
