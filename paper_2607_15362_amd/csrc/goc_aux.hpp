// goc_aux.hpp -- once-per-run and read-out kernels: metric precompute,
// initial state, slot <-> population conversion, fields and global sums.
// One thread per node; none of these is on the per-step path.
#pragma once

#include "goc_step.hpp"

namespace goc {

// (a) Metric precompute in FP64: theta = (dh/dxi) / h^2 (Sec. 2.1, diagonal
// elements on a straight grid) and the block minima of h for q (Sec. 3.2.1).
__global__ void metric_kernel(const double* __restrict__ h, const double* __restrict__ dh,
                              double* __restrict__ th, int n, double* __restrict__ block_min)
{
    __shared__ double smin[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 1e300;
    if (i < n) {
        th[i] = dh[i] / (h[i] * h[i]);
        v = h[i];
    }
    smin[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) block_min[blockIdx.x] = smin[0];
}

// Per-node codec context (one column).
template <class S, class T>
__device__ inline RowCtx<S, T> node_ctx(const RunDesc& d, const Pools<S, typename ForceOf<S>::type>& pl,
                                        int col, Lane& L)
{
    RowCtx<S, T> c{d, pl, d.f_off, d.F_off, d.metric_off_y, T(d.rho0), T(d.cs2), T(1), T(1), T(1), {}};
    const int64_t mx = d.metric_off_x;
    L.col = col;
    L.cvalid = true;
    L.own = true;
    c.h1c = T(pl.h1[mx + col]);
    if constexpr (Store<S>::dev) {
        const int cm = d.bc_x == 0 ? (col + d.nx - 1) % d.nx : max(col - 1, 0);
        const int cp = d.bc_x == 0 ? (col + 1) % d.nx : min(col + 1, d.nx - 1);
        c.h1m1 = T(pl.h1[mx + cm]);
        c.h1p1 = T(pl.h1[mx + cp]);
        for (int k = 0; k < 4; ++k) c.sinv[k] = T(1.0 / d.sc[k]);
    }
    return c;
}

// Destination slot of population a arriving at node (i, j): the slot its
// pull reads (inverse of the gather of the step kernel).
__device__ inline void slot_of(const RunDesc& d, int i, int j, int a, int& si, int& sj, int& pa)
{
    si = i - ex_(a);
    sj = j - ey_(a);
    pa = a;
    bool wall = false;
    if (si < 0 || si >= d.nx) {
        if (d.bc_x == 0) si = si < 0 ? si + d.nx : si - d.nx;
        else wall = true;
    }
    if (sj < 0 || sj >= d.ny) {
        if (d.bc_y == 0) sj = sj < 0 ? sj + d.ny : sj - d.ny;
        else wall = true;
    }
    if (wall) { si = i; sj = j; pa = opp_(a); }
}

template <class S, class T>
__device__ inline void put_slot(const RunDesc& d, const Pools<S, typename ForceOf<S>::type>& pl, S* buf,
                                int64_t off, int si, int sj, int pa, T v, bool mhd_plane, int ci)
{
    T rest = T(0), s = T(1);
    if constexpr (Store<S>::dev) {
        const T h1 = T(pl.h1[d.metric_off_x + si]);
        const T h2 = T(pl.h2[d.metric_off_y + sj]);
        if (!mhd_plane) {
            rest = rest_pop<T>(pa, h1, h2, T(d.rho0), T(d.cs2));
            s = T(d.sc[cls_(pa)]);
        } else {
            const T W = pa % kM == 0 ? T(1.0 - 2.0 * d.csm2) : T(0.5 * d.csm2);
            rest = ci == 1 ? W * h1 * h2 * T(d.B0) : T(0);
            s = T(d.scg);
        }
    }
    Store<S>::st(buf, off + (int64_t)pa * d.plane + (int64_t)sj * d.pitch + si, v, rest, s);
}

// Initial state of App. C from node fields (rho, U1, U2), FP64 inputs
// [ny][nx] (nullptr: rest state rho0, U = 0): raw equilibria of Sec. 3 with
// the corrections of Sec. 5 (finite-difference gradients of the fields),
// f = P^-1 m, scattered to the slots; D2Q5: g = g^eq(0) with B = (0, B0);
// lagged force zero.
template <class S>
__global__ void init_kernel(const RunDesc* __restrict__ runs, int run, Pools<S, typename ForceOf<S>::type> pl,
                            const double* __restrict__ rho_in, const double* __restrict__ u1_in,
                            const double* __restrict__ u2_in)
{
    using T = typename ComputeOf<S>::type;
    using FT = typename ForceOf<S>::type;
    const RunDesc& d = runs[run];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const NodeParams<T> p = node_params<T>(d);
    const T h1 = T(pl.h1[d.metric_off_x + i]), h2 = T(pl.h2[d.metric_off_y + j]);
    const T th11 = T(pl.th11[d.metric_off_x + i]), th22 = T(pl.th22[d.metric_off_y + j]);
    auto at = [&](const double* a, int ii, int jj) -> T {
        return T(a[(int64_t)jj * d.nx + ii]);
    };
    T rho = T(d.rho0), U1 = T(0), U2 = T(0), d1U1 = T(0), d2U2 = T(0), d1r = T(0), d2r = T(0);
    if (rho_in) {
        rho = at(rho_in, i, j);
        U1 = at(u1_in, i, j);
        U2 = at(u2_in, i, j);
        // second-order differences: central, wrapped when periodic, one-sided at walls
        auto fdx = [&](const double* a) -> T {
            if (d.bc_x == 0) return T(0.5) * (at(a, (i + 1) % d.nx, j) - at(a, (i + d.nx - 1) % d.nx, j));
            if (i == 0) return T(0.5) * (T(-3) * at(a, 0, j) + T(4) * at(a, 1, j) - at(a, 2, j));
            if (i == d.nx - 1)
                return T(0.5) * (T(3) * at(a, i, j) - T(4) * at(a, i - 1, j) + at(a, i - 2, j));
            return T(0.5) * (at(a, i + 1, j) - at(a, i - 1, j));
        };
        auto fdy = [&](const double* a) -> T {
            if (d.bc_y == 0) return T(0.5) * (at(a, i, (j + 1) % d.ny) - at(a, i, (j + d.ny - 1) % d.ny));
            if (j == 0) return T(0.5) * (T(-3) * at(a, i, 0) + T(4) * at(a, i, 1) - at(a, i, 2));
            if (j == d.ny - 1)
                return T(0.5) * (T(3) * at(a, i, j) - T(4) * at(a, i, j - 1) + at(a, i, j - 2));
            return T(0.5) * (at(a, i, j + 1) - at(a, i, j - 1));
        };
        d1U1 = fdx(u1_in);
        d1r = fdx(rho_in);
        d2U2 = fdy(u2_in);
        d2r = fdy(rho_in);
    }
    T F1, F2, n3, n4;
    force_and_corrections<T>(p, h1, h2, th11, th22, rho, U1, U2, d1U1, d2U2, d1r, d2r, p.Fx1, p.Fx2,
                             F1, F2, n3, n4);
    const T P = rho * p.cs2, r21 = h2 / h1, r12 = h1 / h2;
    const T k2s = r21 * rho * U1 * U1 + r12 * rho * U2 * U2 + (r21 + r12) * P + n3;
    const T k2d = r21 * rho * U1 * U1 - r12 * rho * U2 * U2 + (r21 - r12) * P + n4;
    const T m00 = h1 * h2 * rho, m10 = h2 * rho * U1, m01 = h1 * rho * U2;
    const T m20 = T(0.5) * (k2s + k2d), m02 = T(0.5) * (k2s - k2d);
    const T m11 = rho * U1 * U2;
    const T m21 = rho * (p.cs2 + U1 * U1) * U2 / h1;
    const T m12 = rho * (p.cs2 + U2 * U2) * U1 / h2;
    const T m22 = rho * p.cs2 * p.cs2 + rho * p.cs2 * (U1 * U1 + U2 * U2) + rho * U1 * U1 * U2 * U2;
    T f[kQ];
    f[0] = m00 - m20 - m02 + m22;
    f[1] = T(0.5) * (m10 + m20 - m12 - m22);
    f[2] = T(0.5) * (m01 + m02 - m21 - m22);
    f[3] = T(0.5) * (-m10 + m20 + m12 - m22);
    f[4] = T(0.5) * (-m01 + m02 + m21 - m22);
    f[5] = T(0.25) * (m11 + m21 + m12 + m22);
    f[6] = T(0.25) * (-m11 + m21 - m12 + m22);
    f[7] = T(0.25) * (m11 - m21 - m12 + m22);
    f[8] = T(0.25) * (-m11 - m21 + m12 + m22);
    for (int a = 0; a < kQ; ++a) {
        int si, sj, pa;
        slot_of(d, i, j, a, si, sj, pa);
        put_slot<S, T>(d, pl, pl.fout, d.f_off, si, sj, pa, f[a], false, 0);
    }
    const int64_t n = (int64_t)j * d.pitch + i;
    pl.Fout[d.F_off + n] = FT(0);
    pl.Fout[d.F_off + n + d.plane] = FT(0);
    if (d.mhd) {
        const T B[2] = {T(0), p.B0};
        const T U[2] = {U1, U2};
        const T hh = h1 * h2;
        for (int ci = 0; ci < 2; ++ci) {
            const T A1 = U[0] * B[ci] - B[0] * U[ci];
            const T A2 = U[1] * B[ci] - B[1] * U[ci];
            for (int a = 0; a < kM; ++a) {
                const T W = a == 0 ? p.W0 : p.W1;
                const T g = W * (hh * B[ci] + (T(ex_(a)) * h2 * A1 + T(ey_(a)) * h1 * A2) * p.inv_csm2);
                int si, sj, pa;
                slot_of(d, i, j, a, si, sj, pa);
                put_slot<S, T>(d, pl, pl.gout, d.g_off, si, sj, ci * kM + pa, g, true, ci);
            }
        }
    }
}

// Post-stream populations (gather) or their inverse (scatter), FP64 node
// arrays f[9][ny][nx], F[2][ny][nx], g[10][ny][nx].
template <class S>
__global__ void gather_kernel(const RunDesc* __restrict__ runs, int run, Pools<S, typename ForceOf<S>::type> pl,
                              double* __restrict__ f, double* __restrict__ F, double* __restrict__ g)
{
    using T = typename ComputeOf<S>::type;
    const RunDesc& d = runs[run];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    Lane L;
    RowCtx<S, T> c = node_ctx<S, T>(d, pl, i, L);
    T fl[kQ];
    pull9<S, T>(c, L, j, fl);
    const int64_t N = (int64_t)d.nx * d.ny, o = (int64_t)j * d.nx + i;
    for (int a = 0; a < kQ; ++a) f[a * N + o] = double(fl[a]);
    const int64_t n = (int64_t)j * d.pitch + i;
    F[o] = double(pl.Fin[d.F_off + n]);
    F[N + o] = double(pl.Fin[d.F_off + n + d.plane]);
    if (d.mhd && g) {
        for (int ci = 0; ci < 2; ++ci)
            for (int a = 0; a < kM; ++a) {
                int si, sj, pa;
                slot_of(d, i, j, a, si, sj, pa);
                const int plane = ci * kM + pa;
                T rest = T(0), inv = T(1);
                if constexpr (Store<S>::dev) {
                    const T W = pa == 0 ? T(1.0 - 2.0 * d.csm2) : T(0.5 * d.csm2);
                    rest = ci == 1 ? W * T(pl.h1[d.metric_off_x + si]) * T(pl.h2[d.metric_off_y + sj]) * T(d.B0) : T(0);
                    inv = T(1.0 / d.scg);
                }
                g[(ci * kM + a) * N + o] = double(Store<S>::ld(
                    pl.gin, d.g_off + plane * d.plane + (int64_t)sj * d.pitch + si, rest, inv));
            }
    }
}

template <class S>
__global__ void scatter_kernel(const RunDesc* __restrict__ runs, int run, Pools<S, typename ForceOf<S>::type> pl,
                               const double* __restrict__ f, const double* __restrict__ F,
                               const double* __restrict__ g)
{
    using T = typename ComputeOf<S>::type;
    using FT = typename ForceOf<S>::type;
    const RunDesc& d = runs[run];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const int64_t N = (int64_t)d.nx * d.ny, o = (int64_t)j * d.nx + i;
    for (int a = 0; a < kQ; ++a) {
        int si, sj, pa;
        slot_of(d, i, j, a, si, sj, pa);
        put_slot<S, T>(d, pl, pl.fout, d.f_off, si, sj, pa, T(f[a * N + o]), false, 0);
    }
    const int64_t n = (int64_t)j * d.pitch + i;
    pl.Fout[d.F_off + n] = FT(F[o]);
    pl.Fout[d.F_off + n + d.plane] = FT(F[N + o]);
    if (d.mhd && g) {
        for (int ci = 0; ci < 2; ++ci)
            for (int a = 0; a < kM; ++a) {
                int si, sj, pa;
                slot_of(d, i, j, a, si, sj, pa);
                put_slot<S, T>(d, pl, pl.gout, d.g_off, si, sj, ci * kM + pa, T(g[(ci * kM + a) * N + o]),
                               true, ci);
            }
    }
}

// Hydrodynamic and magnetic fields of the current state (FP64 outputs).
template <class S>
__global__ void fields_kernel(const RunDesc* __restrict__ runs, int run, Pools<S, typename ForceOf<S>::type> pl,
                              double* __restrict__ rho_o, double* __restrict__ u_o, double* __restrict__ B_o)
{
    using T = typename ComputeOf<S>::type;
    const RunDesc& d = runs[run];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    Lane L;
    RowCtx<S, T> c = node_ctx<S, T>(d, pl, i, L);
    T fl[kQ], rho, U1, U2;
    pull9<S, T>(c, L, j, fl);
    const T h2 = T(pl.h2[d.metric_off_y + j]);
    row_moments<S, T>(c, L, j, fl, h2, rho, U1, U2);
    const int64_t N = (int64_t)d.nx * d.ny, o = (int64_t)j * d.nx + i;
    if (rho_o) rho_o[o] = double(rho);
    if (u_o) {
        u_o[o] = double(U1);
        u_o[N + o] = double(U2);
    }
    if (d.mhd && B_o) {
        T S2[2] = {T(0), T(0)};
        for (int ci = 0; ci < 2; ++ci)
            for (int a = 0; a < kM; ++a) {
                int si, sj, pa;
                slot_of(d, i, j, a, si, sj, pa);
                T rest = T(0), inv = T(1);
                if constexpr (Store<S>::dev) {
                    const T W = pa == 0 ? T(1.0 - 2.0 * d.csm2) : T(0.5 * d.csm2);
                    rest = ci == 1 ? W * T(pl.h1[d.metric_off_x + si]) * T(pl.h2[d.metric_off_y + sj]) * T(d.B0) : T(0);
                    inv = T(1.0 / d.scg);
                }
                S2[ci] += Store<S>::ld(pl.gin, d.g_off + (ci * kM + pa) * d.plane + (int64_t)sj * d.pitch + si,
                                       rest, inv);
            }
        const T ihh = T(1) / (c.h1c * h2);
        B_o[o] = double(S2[0] * ihh);
        B_o[N + o] = double(S2[1] * ihh);
    }
}

// Global sums (FP64 accumulation), one partial per work-group of 256 nodes:
// [0] sum f, [1] sum h2 rho U1, [2] sum h1 rho U2, [3] sum h1 h2 B1,
// [4] sum h1 h2 B2, [5] max |U|, [6] non-finite count.
constexpr int kDiag = 7;
template <class S>
__global__ void diag_kernel(const RunDesc* __restrict__ runs, int run, Pools<S, typename ForceOf<S>::type> pl,
                            double* __restrict__ part)
{
    using T = typename ComputeOf<S>::type;
    __shared__ double sh[kDiag][256];
    const RunDesc& d = runs[run];
    const int64_t N = (int64_t)d.nx * d.ny;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[kDiag] = {0, 0, 0, 0, 0, 0, 0};
    if (idx < N) {
        const int i = (int)(idx % d.nx), j = (int)(idx / d.nx);
        Lane L;
        RowCtx<S, T> c = node_ctx<S, T>(d, pl, i, L);
        T fl[kQ], rho, U1, U2;
        pull9<S, T>(c, L, j, fl);
        const T h2 = T(pl.h2[d.metric_off_y + j]);
        row_moments<S, T>(c, L, j, fl, h2, rho, U1, U2);
        double m = 0;
        int bad = 0;
        for (int a = 0; a < kQ; ++a) {
            m += double(fl[a]);
            bad += isfinite(double(fl[a])) ? 0 : 1;
        }
        v[0] = m;
        v[1] = double(h2) * double(rho) * double(U1);
        v[2] = double(c.h1c) * double(rho) * double(U2);
        if (d.mhd) {
            for (int ci = 0; ci < 2; ++ci) {
                double s = 0;
                for (int a = 0; a < kM; ++a) {
                    int si, sj, pa;
                    slot_of(d, i, j, a, si, sj, pa);
                    T rest = T(0), inv = T(1);
                    if constexpr (Store<S>::dev) {
                        const T W = pa == 0 ? T(1.0 - 2.0 * d.csm2) : T(0.5 * d.csm2);
                        rest = ci == 1 ? W * T(pl.h1[d.metric_off_x + si]) * T(pl.h2[d.metric_off_y + sj]) * T(d.B0) : T(0);
                        inv = T(1.0 / d.scg);
                    }
                    const double gv = double(Store<S>::ld(
                        pl.gin, d.g_off + (ci * kM + pa) * d.plane + (int64_t)sj * d.pitch + si, rest, inv));
                    s += gv;
                    bad += isfinite(gv) ? 0 : 1;
                }
                v[3 + ci] = s;
            }
        }
        v[5] = sqrt(double(U1) * double(U1) + double(U2) * double(U2));
        if (!isfinite(v[5])) { v[5] = 0; bad += 1; }
        v[6] = bad;
    }
    for (int k = 0; k < kDiag; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < kDiag; ++k) {
                if (k == 5) sh[k][threadIdx.x] = fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + s]);
                else sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < kDiag; ++k) part[(int64_t)blockIdx.x * kDiag + k] = sh[k][0];
}

// Second pass over the partials (one work-group), fixed order: deterministic.
__global__ void diag_final_kernel(const double* __restrict__ part, int nparts, double* __restrict__ out)
{
    __shared__ double sh[kDiag][256];
    double v[kDiag] = {0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x)
        for (int k = 0; k < kDiag; ++k) {
            const double x = part[(int64_t)b * kDiag + k];
            v[k] = (k == 5) ? fmax(v[k], x) : v[k] + x;
        }
    for (int k = 0; k < kDiag; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < kDiag; ++k) {
                if (k == 5) sh[k][threadIdx.x] = fmax(sh[k][threadIdx.x], sh[k][threadIdx.x + s]);
                else sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < kDiag; ++k) out[k] = sh[k][0];
}

}  // namespace goc
