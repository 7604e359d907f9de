// goc_step.hpp -- the fused time-step kernel.
#pragma once

#include "goc_device.hpp"

namespace goc {

// Compute type of a storage type.
template <class S> struct ComputeOf { using type = float; };
template <> struct ComputeOf<double> { using type = double; };
// Storage type of the lagged force.
template <class S> struct ForceOf { using type = float; };
template <> struct ForceOf<double> { using type = double; };

// Column geometry of one lane: the node column, its two neighbours (wrapped
// when periodic) and whether they lie beyond a wall.
struct LaneCol {
    int col, cm, cp;
    bool valid;     // col inside the grid
    bool wm, wp;    // -xi1 / +xi1 neighbour beyond a wall
};

__device__ inline LaneCol lane_col(const RunDesc& d, int craw)
{
    LaneCol L;
    if (d.bc_x == 0) {
        L.col = ((craw % d.nx) + d.nx) % d.nx;
        L.valid = true;
        L.cm = L.col == 0 ? d.nx - 1 : L.col - 1;
        L.cp = L.col == d.nx - 1 ? 0 : L.col + 1;
        L.wm = L.wp = false;
    } else {
        L.col = craw;
        L.valid = craw >= 0 && craw < d.nx;
        L.cm = craw - 1;
        L.cp = craw + 1;
        L.wm = craw == 0;
        L.wp = craw == d.nx - 1;
    }
    return L;
}

// Row geometry: a row, its neighbours (wrapped when periodic) and walls.
struct RowGeo {
    int r, rm, rp;
    bool wm, wp;
};

__device__ inline RowGeo row_geo(const RunDesc& d, int r)
{
    RowGeo G;
    G.r = r;
    if (d.bc_y == 0) {
        G.rm = r == 0 ? d.ny - 1 : r - 1;
        G.rp = r == d.ny - 1 ? 0 : r + 1;
        G.wm = G.wp = false;
    } else {
        G.rm = r - 1;
        G.rp = r + 1;
        G.wm = r == 0;
        G.wp = r == d.ny - 1;
    }
    return G;
}

__device__ inline bool row_ok(const RunDesc& d, int r) { return d.bc_y == 0 || (r >= 0 && r < d.ny); }
__device__ inline int row_wrap(const RunDesc& d, int r) { return d.bc_y == 0 ? (r % d.ny + d.ny) % d.ny : r; }

// Element offset (within a run's pool region) of the slot pulled by
// direction a into node (L.col, G.r): slot(a, x - e_a) in the interior,
// slot(opp(a), x) through a wall.
__device__ inline int64_t pull_index(const RunDesc& d, const LaneCol& L, const RowGeo& G, int a)
{
    const int ex = ex_(a), ey = ey_(a);
    const bool wx = (ex > 0 && L.wm) || (ex < 0 && L.wp);
    const bool wy = (ey > 0 && G.wm) || (ey < 0 && G.wp);
    int sx = ex > 0 ? L.cm : (ex < 0 ? L.cp : L.col);
    int sy = ey > 0 ? G.rm : (ey < 0 ? G.rp : G.r);
    int pa = a;
    if (wx || wy) {
        sx = L.col;
        sy = G.r;
        pa = opp_(a);
    }
    return (int64_t)pa * d.plane + (int64_t)sy * d.pitch + sx;
}

// Pull the nine deviations of node (col, r).
template <class S, class T>
__device__ inline void pull9(const RunDesc& d, const S* __restrict__ fin, const LaneCol& L, const RowGeo& G,
                             const T* sinv, T* f)
{
    const S* base = fin + d.f_off;
#pragma unroll
    for (int a = 0; a < kQ; ++a)
        f[a] = L.valid ? T(Store<S>::ld(base, pull_index(d, L, G, a), sinv[cls_(a)])) : T(0);
}

// Moments of a pulled row: the density deviation dr = rho - rho0 =
// dm00/(h1 h2) (kept as a deviation, so FP32 does not round it against
// rho0), U1 = (dm10 + F1/2)/(rho h2), U2 = (dm01 + F2/2)/(rho h1) with the
// lagged effective force Fp (App. E step 7), which is returned too.
template <class FT, class T>
__device__ inline void row_moments(const RunDesc& d, const FT* __restrict__ Fin, const LaneCol& L, int r,
                                   const T* f, T rho0, T ih1, T ih2, T& dr, T& U1, T& U2, T& Fp1, T& Fp2)
{
    const T m00 = f[0] + f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    const T m10 = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
    const T m01 = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
    Fp1 = T(0);
    Fp2 = T(0);
    if (L.valid) {
        const int64_t n = d.F_off + (int64_t)r * d.pitch + L.col;
        Fp1 = T(Fin[n]);
        Fp2 = T(Fin[n + d.plane]);
    }
    dr = m00 * ih1 * ih2;
    const T irho = recip_sum(rho0, dr);
    U1 = (m10 + T(0.5) * Fp1) * ih2 * irho;
    U2 = (m01 + T(0.5) * Fp2) * ih1 * irho;
}

// Rounding draws of a node's populations: the node hash hn times distinct
// odd multipliers (D2Q9 populations 0-8, then the ten D2Q5 populations).
__device__ inline uint32_t pop_draw(uint32_t hn, int a) { return hn * (0x9E3779B1u * uint32_t(2 * a + 1)); }

// One time step for every run of the launch.
//   grid.x = total work-groups, block = 64 (one wave).
//   block_run[b]: run of work-group b.
//   step_ctr[0] + k: the step's index in the sequence of rounding draws.
template <class S, bool MHD>
__global__ void __launch_bounds__(kWave) step_kernel(const RunDesc* __restrict__ runs,
                                                     const int32_t* __restrict__ block_run,
                                                     Pools<S, typename ForceOf<S>::type> pl,
                                                     const uint32_t* __restrict__ step_ctr, int k)
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
    const uint32_t seed = mix32(step_ctr[0] + uint32_t(k));

    // lane geometry and column metric
    const int lb = lane_base(d.nx, d.bc_x, strip);
    const int craw = lb + lane;
    const LaneCol L = lane_col(d, craw);
    const int x0 = strip * kOwn;
    const int x1 = min(x0 + kOwn, d.nx);
    const bool own = lane >= 1 && lane <= kWave - 2 && craw >= x0 && craw < x1;
    const bool xwall_lo = d.bc_x != 0 && L.col == 0;
    const bool xwall_hi = d.bc_x != 0 && L.col == d.nx - 1;
    T h1 = T(1), ih1 = T(1), th11 = T(0), a1p = T(0), a1m = T(0), b1p = T(0), b1m = T(0);
    if (L.valid) {
        const double* ct = pl.col + (d.col_off + L.col) * kTab;
        h1 = T(ct[T_H]);
        ih1 = T(ct[T_IH]);
        th11 = T(ct[T_TH]);
        a1p = T(ct[T_AP]);
        a1m = T(ct[T_AM]);
        b1p = T(ct[T_BP]);
        b1m = T(ct[T_BM]);
    }
    T sinv[4], sfw[4], sginv = T(1), sgw = T(1);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sinv[k] = Store<S>::scaled ? T(1.0 / d.sc[k]) : T(1);
        sfw[k] = Store<S>::scaled ? T(d.sc[k]) : T(1);
    }
    if (Store<S>::scaled) {
        sginv = T(1.0 / d.scg);
        sgw = T(d.scg);
    }
    const double* rowtab = pl.row + d.row_off * kTab;
    auto ih2_of = [&](int r) { return T(rowtab[r * kTab + T_IH]); };

    int y0, y1;
    seg_rows(d.ny, d.segs, seg, y0, y1);

    // Window of row moments: rows j-2, j-1, j, j+1 (rho - rho0, U2) and row
    // j (U1, f).
    T wr[4] = {T(0), T(0), T(0), T(0)}, wu[4] = {T(0), T(0), T(0), T(0)};
    T fc[kQ], fn[kQ];
    T U1c = T(0), U1n = T(0);
    // lagged force of rows j and j+1: the first central moments relax by
    // exactly half of it (see cm_collide)
    T Fpc1, Fpc2, Fpn1 = T(0), Fpn2 = T(0);
    if (row_ok(d, y0 - 1)) {
        const int r = row_wrap(d, y0 - 1);
        T ft[kQ], u1, q1, q2;
        pull9<S, T>(d, pl.fin, L, row_geo(d, r), sinv, ft);
        row_moments<FT, T>(d, pl.Fin, L, r, ft, p.rho0, ih1, ih2_of(r), wr[1], u1, wu[1], q1, q2);
    }
    pull9<S, T>(d, pl.fin, L, row_geo(d, y0), sinv, fc);
    row_moments<FT, T>(d, pl.Fin, L, y0, fc, p.rho0, ih1, ih2_of(y0), wr[2], U1c, wu[2], Fpc1, Fpc2);

    const int64_t plane = d.plane;
    for (int j = y0; j < y1; ++j) {
        if (row_ok(d, j + 1)) {
            const int r = row_wrap(d, j + 1);
            pull9<S, T>(d, pl.fin, L, row_geo(d, r), sinv, fn);
            row_moments<FT, T>(d, pl.Fin, L, r, fn, p.rho0, ih1, ih2_of(r), wr[3], U1n, wu[3], Fpn1, Fpn2);
        }
        const double* rt = rowtab + j * kTab;
        NodeMetric<T> g;
        g.h1 = h1;
        g.ih1 = ih1;
        g.th11 = th11;
        g.h2 = T(rt[T_H]);
        g.ih2 = T(rt[T_IH]);
        g.th22 = T(rt[T_TH]);
        // finite differences along xi2 (one-sided next to walls)
        T d2U2, d2r;
        if (d.bc_y != 0 && j == 0) {
            T f2[kQ], r2, u12, u22, q1, q2;
            pull9<S, T>(d, pl.fin, L, row_geo(d, 2), sinv, f2);
            row_moments<FT, T>(d, pl.Fin, L, 2, f2, p.rho0, ih1, ih2_of(2), r2, u12, u22, q1, q2);
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
        const T drho = wr[2], rho = p.rho0 + drho, U2 = wu[2], U1 = U1c;
        const int lm1 = max(lane - 1, 0), lp1 = min(lane + 1, kWave - 1);
        const int lm2 = max(lane - 2, 0), lp2 = min(lane + 2, kWave - 1);
        const T Um1 = shfl(U1, lm1), Up1 = shfl(U1, lp1), Um2 = shfl(U1, lm2), Up2 = shfl(U1, lp2);
        const T rm1 = shfl(drho, lm1), rp1 = shfl(drho, lp1), rm2 = shfl(drho, lm2), rp2 = shfl(drho, lp2);
        T d1U1, d1r;
        if (xwall_lo) {
            d1U1 = T(0.5) * (T(-3) * U1 + T(4) * Up1 - Up2);
            d1r = T(0.5) * (T(-3) * drho + T(4) * rp1 - rp2);
        } else if (xwall_hi) {
            d1U1 = T(0.5) * (T(3) * U1 - T(4) * Um1 + Um2);
            d1r = T(0.5) * (T(3) * drho - T(4) * rm1 + rm2);
        } else {
            d1U1 = T(0.5) * (Up1 - Um1);
            d1r = T(0.5) * (rp1 - rm1);
        }

        // App. G: magnetic field, local derivatives, Lorentz force, collision
        T Fx1 = p.Fx1, Fx2 = p.Fx2;
        T dg[2][kM], dgi[2][kM];
        const bool mhd_run = MHD && d.mhd;   // a batch may mix MHD and plain runs
        const RowGeo Gj = row_geo(d, j);
        if (mhd_run) {
            const S* gb = pl.gin + d.g_off;
#pragma unroll
            for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                for (int a = 0; a < kM; ++a)
                    dg[ci][a] = L.valid ? T(Store<S>::ld(gb, ci * kM * plane + pull_index(d, L, Gj, a), sginv))
                                        : T(0);
            T B1, B2, FL1, FL2;
            mie_node<T>(p, g, dg, U1, U2, B1, B2, FL1, FL2, dgi);
            Fx1 += FL1;
            Fx2 += FL2;
        }

        T F1, F2, n3, n4, inc[kQ];
        force_and_corrections<T>(p, g, rho, drho, U1, U2, d1U1, d2U2, d1r, d2r, Fx1, Fx2, F1, F2, n3, n4);
        cm_collide<T>(p, g, raw_dev<T>(fc), rho, drho, U1, U2, Fpc1, Fpc2, F1, F2, n3, n4, inc);

        if (own) {
            // inc holds the collision increments; the writer adds the
            // rest-state offsets of the interior axis slots (the reader is
            // the neighbour; its rest state differs through the metric)
            const T a2p = T(rt[T_AP]), a2m = T(rt[T_AM]);
            inc[1] += g.h2 * a1p;
            inc[3] += g.h2 * a1m;
            inc[2] += g.h1 * a2p;
            inc[4] += g.h1 * a2m;
            // writer-side momentum-augmented bounce-back of App. C for
            // populations leaving through a moving y-wall
            if (Gj.wp && d.uw_hi != 0.0) {
                const T cw = rho * p.cs2 * T(d.uw_hi) / (T(2) * T(d.hw_hi));
                // slot 5 is read back as f7, slot 6 as f8: f7 = ft5 - cw, f8 = ft6 + cw
                if (d.lid_corners || !xwall_hi) inc[5] -= cw;
                if (d.lid_corners || !xwall_lo) inc[6] += cw;
            }
            if (Gj.wm && d.uw_lo != 0.0) {
                const T cw = rho * p.cs2 * T(d.uw_lo) / (T(2) * T(d.hw_lo));
                // slot 7 is read back as f5, slot 8 as f6: f5 = ft7 + cw, f6 = ft8 - cw
                if (d.lid_corners || !xwall_lo) inc[7] += cw;
                if (d.lid_corners || !xwall_hi) inc[8] -= cw;
            }
            const int64_t nn = (int64_t)j * d.pitch + L.col;
            const uint32_t hn = mix32(uint32_t(d.f_off + nn) ^ seed);
            S* fo = pl.fout + d.f_off + nn;
#pragma unroll
            for (int a = 0; a < kQ; ++a) Store<S>::st_sr(fo, a * plane, fc[a], inc[a], sfw[cls_(a)], pop_draw(hn, a));
            pl.Fout[d.F_off + nn] = FT(F1);
            pl.Fout[d.F_off + nn + plane] = FT(F2);
            if (mhd_run) {
                // stored value = base + increment; anti-bounce-back slots
                // negate the post-collision value
                const T b2p = T(rt[T_BP]), b2m = T(rt[T_BM]);
                const T hh = g.h1 * g.h2;
#pragma unroll
                for (int a = 1; a < kM; ++a) {
                    const int ex = ex_(a), ey = ey_(a);
                    const bool wx = (ex > 0 && L.wp) || (ex < 0 && L.wm);
                    const bool wy = (ey > 0 && Gj.wp) || (ey < 0 && Gj.wm);
                    if (wx || wy) {
                        // anti-bounce-back of App. G: the reader (this node) sees
                        // -g~ + 2 W h_wall B_wall with B_wall = (0, B0)
                        const T hwall = wy ? g.h1 * T(ey < 0 ? d.hw_lo : d.hw_hi)
                                           : T(ex < 0 ? d.h1w_lo : d.h1w_hi) * g.h2;
                        dg[0][a] = -dg[0][a];
                        dgi[0][a] = -dgi[0][a];
                        dg[1][a] = -dg[1][a];
                        dgi[1][a] = -dgi[1][a] + T(2) * p.W1 * p.B0 * (hwall - hh);
                    } else {
                        dgi[1][a] += a == 1 ? g.h2 * b1p : a == 3 ? g.h2 * b1m : a == 2 ? g.h1 * b2p : g.h1 * b2m;
                    }
                }
                S* go = pl.gout + d.g_off + nn;
#pragma unroll
                for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                    for (int a = 0; a < kM; ++a)
                        Store<S>::st_sr(go, (ci * kM + a) * plane, dg[ci][a], dgi[ci][a], sgw,
                                        pop_draw(hn, kQ + ci * kM + a));
            }
        }
        // shift the window
        wr[0] = wr[1]; wu[0] = wu[1];
        wr[1] = wr[2]; wu[1] = wu[2];
        wr[2] = wr[3]; wu[2] = wu[3];
        U1c = U1n;
        Fpc1 = Fpn1;
        Fpc2 = Fpn2;
#pragma unroll
        for (int a = 0; a < kQ; ++a) fc[a] = fn[a];
    }
}

}  // namespace goc
