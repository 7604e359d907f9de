// goc_step.hpp -- the fused time-step kernel and the state conversion kernels.
#pragma once

#include "goc_device.hpp"

namespace goc {

// Compute type of a storage type.
template <class S> struct ComputeOf { using type = float; };
template <> struct ComputeOf<double> { using type = double; };
// Storage type of the lagged force.
template <class S> struct ForceOf { using type = float; };
template <> struct ForceOf<double> { using type = double; };

// Per-lane geometry of one work-group.
struct Lane {
    int col;        // column (wrapped for periodic x); valid iff cvalid
    bool cvalid;
    bool own;       // this lane writes its column
    int colm1, colp1;  // neighbour columns for the rest state of the 16-bit codec
};

template <class S, class T>
struct RowCtx {
    const RunDesc& d;
    const Pools<S, typename ForceOf<S>::type>& pl;
    int64_t base;     // element offset of this run's f plane 0
    int64_t Fbase;    // element offset of this run's force plane 0
    int64_t moff;     // element offset of this run's row metric
    T rho0, cs2;
    T h1c, h1m1, h1p1;   // h1 at the lane's column and its neighbours (16-bit codec)
    T sinv[4];
};

// Row index wrap / validity.
__device__ inline bool row_ok(const RunDesc& d, int r) { return d.bc_y == 0 || (r >= 0 && r < d.ny); }
__device__ inline int row_wrap(const RunDesc& d, int r) { return d.bc_y == 0 ? (r % d.ny + d.ny) % d.ny : r; }

// Pull the nine pre-collision populations of node (col, r) (App. E step 6
// as a gather; wall slots were written by the wall-adjacent node itself).
template <class S, class T>
__device__ inline void pull9(const RowCtx<S, T>& c, const Lane& L, int r, T* f)
{
    const RunDesc& d = c.d;
    const int64_t pitch = d.pitch, plane = d.plane;
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        int sx = L.col - ex_(a), sy = r - ey_(a);
        int pa = a;
        bool wall = false;
        if (sx < 0 || sx >= d.nx) {
            if (d.bc_x == 0) sx = sx < 0 ? sx + d.nx : sx - d.nx;
            else wall = true;
        }
        if (sy < 0 || sy >= d.ny) {
            if (d.bc_y == 0) sy = sy < 0 ? sy + d.ny : sy - d.ny;
            else wall = true;
        }
        if (wall) { sx = L.col; sy = r; pa = opp_(a); }
        T rest = T(0), inv = T(1);
        if constexpr (Store<S>::dev) {
            const T h1s = (sx == L.col) ? c.h1c : (ex_(a) > 0 ? c.h1m1 : c.h1p1);
            const T h2s = T(c.pl.h2[c.moff + sy]);
            rest = rest_pop<T>(pa, h1s, h2s, c.rho0, c.cs2);
            inv = c.sinv[cls_(pa)];
        }
        f[a] = L.cvalid ? Store<S>::ld(c.pl.fin, c.base + pa * plane + (int64_t)sy * pitch + sx, rest, inv)
                        : T(0);
    }
}

template <class S>
__device__ inline int64_t node_index(const RunDesc& d, int col, int r) { return (int64_t)r * d.pitch + col; }

// Moments of a pulled row: rho = k00/(h1 h2), U1 = (k10 + F1/2)/(rho h2),
// U2 = (k01 + F2/2)/(rho h1) with the lagged force (App. E step 7).
template <class S, class T>
__device__ inline void row_moments(const RowCtx<S, T>& c, const Lane& L, int r, const T* f, T h2,
                                   T& rho, T& U1, T& U2)
{
    const T m00 = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    const T m10 = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
    const T m01 = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
    T Fp1 = T(0), Fp2 = T(0);
    if (L.cvalid) {
        const int64_t n = c.Fbase + node_index<S>(c.d, L.col, r);
        Fp1 = T(c.pl.Fin[n]);
        Fp2 = T(c.pl.Fin[n + c.d.plane]);
    }
    const T h1 = c.h1c;
    rho = L.cvalid ? m00 / (h1 * h2) : T(1);
    U1 = L.cvalid ? (m10 + T(0.5) * Fp1) / (rho * h2) : T(0);
    U2 = L.cvalid ? (m01 + T(0.5) * Fp2) / (rho * h1) : T(0);
}

// One time step for every run of the launch.
//   grid.x = total work-groups, block = 64 (one wave).
//   block_run[b]: run of work-group b.
template <class S, bool MHD>
__global__ void __launch_bounds__(kWave) step_kernel(const RunDesc* __restrict__ runs,
                                                     const int32_t* __restrict__ block_run,
                                                     Pools<S, typename ForceOf<S>::type> pl)
{
    using T = typename ComputeOf<S>::type;
    using FT = typename ForceOf<S>::type;
    const int run = block_run[blockIdx.x];
    const RunDesc& d = runs[run];
    const int local = blockIdx.x - d.first_block;
    const int strip = local % d.strips;
    const int seg = local / d.strips;
    const int lane = threadIdx.x;
    const NodeParams<T> p = node_params<T>(d);

    // lane geometry
    Lane L;
    const int lb = lane_base(d.nx, d.bc_x, strip);
    const int craw = lb + lane;
    const int x0 = strip * kOwn;
    const int x1 = min(x0 + kOwn, d.nx);
    if (d.bc_x == 0) {
        L.col = ((craw % d.nx) + d.nx) % d.nx;
        L.cvalid = true;
    } else {
        L.col = craw;
        L.cvalid = craw >= 0 && craw < d.nx;
    }
    L.own = lane >= 1 && lane <= kWave - 2 && craw >= x0 && craw < x1;
    const bool xwall_lo = d.bc_x != 0 && L.col == 0;
    const bool xwall_hi = d.bc_x != 0 && L.col == d.nx - 1;

    RowCtx<S, T> c{d, pl, d.f_off, d.F_off, d.metric_off_y, T(d.rho0), T(d.cs2), T(1), T(1), T(1), {}};
    const int64_t mx = d.metric_off_x;
    const T h1 = L.cvalid ? T(pl.h1[mx + L.col]) : T(1);
    const T th11 = L.cvalid ? T(pl.th11[mx + L.col]) : T(0);
    c.h1c = h1;
    if constexpr (Store<S>::dev) {
        const int cm = d.bc_x == 0 ? (L.col + d.nx - 1) % d.nx : max(L.col - 1, 0);
        const int cp = d.bc_x == 0 ? (L.col + 1) % d.nx : min(L.col + 1, d.nx - 1);
        c.h1m1 = L.cvalid ? T(pl.h1[mx + cm]) : T(1);
        c.h1p1 = L.cvalid ? T(pl.h1[mx + cp]) : T(1);
#pragma unroll
        for (int k = 0; k < 4; ++k) c.sinv[k] = T(1.0 / d.sc[k]);
    }

    int y0, y1;
    seg_rows(d.ny, d.segs, seg, y0, y1);

    // Window of row moments: rows j-2, j-1, j, j+1 (rho, U2) and row j (U1, f).
    T wr[4] = {T(1), T(1), T(1), T(1)}, wu[4] = {T(0), T(0), T(0), T(0)};
    T fc[kQ], fn[kQ];
    T U1c = T(0), U1n = T(0);
    auto h2_of = [&](int r) { return T(pl.h2[d.metric_off_y + row_wrap(d, r)]); };
    if (row_ok(d, y0 - 1)) {
        const int r = row_wrap(d, y0 - 1);
        T ft[kQ], u1;
        pull9<S, T>(c, L, r, ft);
        row_moments<S, T>(c, L, r, ft, h2_of(r), wr[1], u1, wu[1]);
    }
    {
        pull9<S, T>(c, L, y0, fc);
        row_moments<S, T>(c, L, y0, fc, h2_of(y0), wr[2], U1c, wu[2]);
    }

    const int64_t plane = d.plane;
    const T Fe1 = p.Fx1, Fe2 = p.Fx2;
    for (int j = y0; j < y1; ++j) {
        if (row_ok(d, j + 1)) {
            const int r = row_wrap(d, j + 1);
            pull9<S, T>(c, L, r, fn);
            row_moments<S, T>(c, L, r, fn, h2_of(r), wr[3], U1n, wu[3]);
        }
        const T h2 = h2_of(j);
        const T th22 = T(pl.th22[d.metric_off_y + j]);
        // finite differences along xi2 (one-sided next to walls)
        T d2U2, d2r;
        if (d.bc_y != 0 && j == 0) {
            T f2[kQ], r2, u12, u22;
            pull9<S, T>(c, L, 2, f2);
            row_moments<S, T>(c, L, 2, f2, h2_of(2), r2, u12, u22);
            d2U2 = T(0.5) * (T(-3) * wu[2] + T(4) * wu[3] - u22);
            d2r = T(0.5) * (T(-3) * wr[2] + T(4) * wr[3] - r2);
        } else if (d.bc_y != 0 && j == d.ny - 1) {
            d2U2 = T(0.5) * (T(3) * wu[2] - T(4) * wu[1] + wu[0]);
            d2r = T(0.5) * (T(3) * wr[2] - T(4) * wr[1] + wr[0]);
        } else {
            d2U2 = T(0.5) * (wu[3] - wu[1]);
            d2r = T(0.5) * (wr[3] - wr[1]);
        }
        // finite differences along xi1 from neighbouring lanes
        const T rho = wr[2], U2 = wu[2], U1 = U1c;
        const int lm1 = max(lane - 1, 0), lp1 = min(lane + 1, kWave - 1);
        const int lm2 = max(lane - 2, 0), lp2 = min(lane + 2, kWave - 1);
        const T Um1 = shfl(U1, lm1), Up1 = shfl(U1, lp1), Um2 = shfl(U1, lm2), Up2 = shfl(U1, lp2);
        const T rm1 = shfl(rho, lm1), rp1 = shfl(rho, lp1), rm2 = shfl(rho, lm2), rp2 = shfl(rho, lp2);
        T d1U1, d1r;
        if (xwall_lo) {
            d1U1 = T(0.5) * (T(-3) * U1 + T(4) * Up1 - Up2);
            d1r = T(0.5) * (T(-3) * rho + T(4) * rp1 - rp2);
        } else if (xwall_hi) {
            d1U1 = T(0.5) * (T(3) * U1 - T(4) * Um1 + Um2);
            d1r = T(0.5) * (T(3) * rho - T(4) * rm1 + rm2);
        } else {
            d1U1 = T(0.5) * (Up1 - Um1);
            d1r = T(0.5) * (rp1 - rm1);
        }

        // App. G: magnetic field, local derivatives, Lorentz force, collision
        T Fx1 = Fe1, Fx2 = Fe2;
        T gt[2][kM];
        const bool mhd_run = MHD && d.mhd;   // a batch may mix MHD and plain runs
        if (mhd_run) {
            T gb[2][kM];
#pragma unroll
            for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                for (int a = 0; a < kM; ++a) {
                    int sx = L.col - ex_(a), sy = j - ey_(a);
                    int pa = a;
                    bool wall = false;
                    if (sx < 0 || sx >= d.nx) {
                        if (d.bc_x == 0) sx = sx < 0 ? sx + d.nx : sx - d.nx;
                        else wall = true;
                    }
                    if (sy < 0 || sy >= d.ny) {
                        if (d.bc_y == 0) sy = sy < 0 ? sy + d.ny : sy - d.ny;
                        else wall = true;
                    }
                    if (wall) { sx = L.col; sy = j; pa = opp_(a); }
                    T rest = T(0), inv = T(1);
                    if constexpr (Store<S>::dev) {
                        const T h1s = (sx == L.col) ? h1 : (ex_(a) > 0 ? c.h1m1 : c.h1p1);
                        const T h2s = T(pl.h2[d.metric_off_y + sy]);
                        rest = (ci == 1 ? (pa == 0 ? p.W0 : p.W1) * h1s * h2s * p.B0 : T(0));
                        inv = T(1.0 / d.scg);
                    }
                    gb[ci][a] = L.cvalid ? Store<S>::ld(pl.gin, d.g_off + (ci * kM + pa) * plane +
                                                                     (int64_t)sy * d.pitch + sx, rest, inv)
                                         : T(0);
                }
            T B1, B2, FL1, FL2;
            mie_node<T>(p, h1, h2, th11, th22, gb, U1, U2, B1, B2, FL1, FL2, gt);
            Fx1 += FL1;
            Fx2 += FL2;
        }

        T F1, F2, n3, n4, ft[kQ];
        force_and_corrections<T>(p, h1, h2, th11, th22, rho, U1, U2, d1U1, d2U2, d1r, d2r, Fx1, Fx2,
                                 F1, F2, n3, n4);
        cm_collide<T>(p, h1, h2, fc, rho, U1, U2, F1, F2, n3, n4, ft);

        if (L.own) {
            // writer-side wall conditions: momentum-augmented bounce-back of
            // App. C for populations leaving through a y-wall
            const bool top = d.bc_y != 0 && j == d.ny - 1;
            const bool bot = d.bc_y != 0 && j == 0;
            if (top && d.uw_hi != 0.0) {
                const T cw = rho * p.cs2 * T(d.uw_hi) / (T(2) * T(d.hw_hi));
                // slot 5 is read back as f7, slot 6 as f8: f7 = ft5 - cw, f8 = ft6 + cw
                if (d.lid_corners || !xwall_hi) ft[5] -= cw;
                if (d.lid_corners || !xwall_lo) ft[6] += cw;
            }
            if (bot && d.uw_lo != 0.0) {
                const T cw = rho * p.cs2 * T(d.uw_lo) / (T(2) * T(d.hw_lo));
                // slot 7 is read back as f5, slot 8 as f6: f5 = ft7 + cw, f6 = ft8 - cw
                if (d.lid_corners || !xwall_lo) ft[7] += cw;
                if (d.lid_corners || !xwall_hi) ft[8] -= cw;
            }
            const int64_t nn = node_index<S>(d, L.col, j);
            const int64_t n = d.f_off + nn;
#pragma unroll
            for (int a = 0; a < kQ; ++a) {
                T rest = T(0), s = T(1);
                if constexpr (Store<S>::dev) {
                    rest = rest_pop<T>(a, h1, h2, c.rho0, c.cs2);
                    s = T(d.sc[cls_(a)]);
                }
                Store<S>::st(pl.fout, n + a * plane, ft[a], rest, s);
            }
            pl.Fout[d.F_off + nn] = FT(F1);
            pl.Fout[d.F_off + nn + plane] = FT(F2);
            if (mhd_run) {
                // anti-bounce-back of App. G for populations leaving through a
                // wall: the reader sees -gt + 2 W h_wall B_wall (B_wall = (0, B0))
#pragma unroll
                for (int a = 1; a < kM; ++a) {
                    const int tx = L.col + ex_(a), ty = j + ey_(a);
                    const bool wx = d.bc_x != 0 && (tx < 0 || tx >= d.nx);
                    const bool wy = d.bc_y != 0 && (ty < 0 || ty >= d.ny);
                    if (wx || wy) {
                        T hwall;
                        if (wy) hwall = h1 * T(ty < 0 ? d.hw_lo : d.hw_hi);
                        else hwall = T(tx < 0 ? d.h1w_lo : d.h1w_hi) * h2;
                        gt[0][a] = -gt[0][a];
                        gt[1][a] = -gt[1][a] + T(2) * p.W1 * hwall * p.B0;
                    }
                }
#pragma unroll
                for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                    for (int a = 0; a < kM; ++a) {
                        T rest = T(0), s = T(1);
                        if constexpr (Store<S>::dev) {
                            rest = ci == 1 ? (a == 0 ? p.W0 : p.W1) * h1 * h2 * p.B0 : T(0);
                            s = T(d.scg);
                        }
                        Store<S>::st(pl.gout, d.g_off + nn + (ci * kM + a) * plane, gt[ci][a], rest, s);
                    }
            }
        }
        // shift the window
        wr[0] = wr[1]; wu[0] = wu[1];
        wr[1] = wr[2]; wu[1] = wu[2];
        wr[2] = wr[3]; wu[2] = wu[3];
        U1c = U1n;
#pragma unroll
        for (int a = 0; a < kQ; ++a) fc[a] = fn[a];
    }
}

}  // namespace goc
