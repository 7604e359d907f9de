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

// Metric table of the compute type: the FP64 tables for FP64 arithmetic,
// their FP32 copy otherwise.
template <class T> __device__ inline const T* table_of(const double* d, const float* f);
template <> __device__ inline const double* table_of<double>(const double* d, const float*) { return d; }
template <> __device__ inline const float* table_of<float>(const double*, const float* f) { return f; }

// Whole-wave lane shifts (DPP wave_shr:1 / wave_shl:1): lane i receives the
// value of lane i - 1 / i + 1, and the edge lane keeps its own.
__device__ inline int dpp_prev(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false); }
__device__ inline int dpp_next(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false); }
__device__ inline float from_prev(float v) { return __int_as_float(dpp_prev(__float_as_int(v))); }
__device__ inline float from_next(float v) { return __int_as_float(dpp_next(__float_as_int(v))); }
__device__ inline double from_prev(double v)
{
    const int lo = dpp_prev(__double2loint(v)), hi = dpp_prev(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ inline double from_next(double v)
{
    const int lo = dpp_next(__double2loint(v)), hi = dpp_next(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// State of one pulled row in the marching window: the raw slots (storage
// type, possibly still in flight), the decoded deviations and the moments.
template <class S, class T, class FT>
struct RowSlot {
    S raw[kQ];
    FT Fr[2];       // lagged force F^(n-1)
    S graw[2][kM];  // D2Q5 slots of the row (MHD)
    T f[kQ];
    T dr, U1, U2, Fp1, Fp2;
};

// Issue the loads of the nine slots pulled into row r (and its lagged
// force).  Interior rows (0 < r < ny - 1): every direction's source row is
// uniform, so the address is a per-(plane, row) base plus the lane's
// constant offset off[a].  Rows 0 and ny - 1 (walls or periodic wrap) take
// the general index.
template <class S, class FT>
__device__ inline void issue_row(const RunDesc& d, const S* __restrict__ fin, const FT* __restrict__ Fin,
                                 const LaneCol& Ls, const int32_t* off, int r, S* raw, FT* Fr)
{
    const S* fb = fin + d.f_off;
    if (r > 0 && r < d.ny - 1) {
#pragma unroll
        for (int a = 0; a < kQ; ++a)
            raw[a] = (fb + (int64_t)a * d.plane + (int64_t)(r - ey_(a)) * d.pitch)[off[a]];
    } else {
        const RowGeo G = row_geo(d, r);
#pragma unroll
        for (int a = 0; a < kQ; ++a) raw[a] = fb[pull_index(d, Ls, G, a)];
    }
    const FT* Fb = Fin + d.F_off + (int64_t)r * d.pitch;
    Fr[0] = Fb[Ls.col];
    Fr[1] = Fb[Ls.col + d.plane];
}

// The same for the ten D2Q5 slots of row r.
template <class S>
__device__ inline void issue_row_g(const RunDesc& d, const S* __restrict__ gin, const LaneCol& Ls,
                                   const int32_t* off, int r, S (*graw)[kM])
{
    const S* gb = gin + d.g_off;
    if (r > 0 && r < d.ny - 1) {
#pragma unroll
        for (int ci = 0; ci < 2; ++ci)
#pragma unroll
            for (int a = 0; a < kM; ++a)
                graw[ci][a] = (gb + (int64_t)(ci * kM + a) * d.plane + (int64_t)(r - ey_(a)) * d.pitch)[off[a]];
    } else {
        const RowGeo G = row_geo(d, r);
#pragma unroll
        for (int ci = 0; ci < 2; ++ci)
#pragma unroll
            for (int a = 0; a < kM; ++a) graw[ci][a] = gb[(int64_t)ci * kM * d.plane + pull_index(d, Ls, G, a)];
    }
}

// Decode a pulled row and form its moments: dr = rho - rho0 = dm00/(h1 h2),
// U1 = (dm10 + F1/2)/(rho h2), U2 = (dm01 + F2/2)/(rho h1) with the lagged
// effective force (App. E step 7).
template <class S, class T, class FT>
__device__ inline void decode_row(RowSlot<S, T, FT>& R, const T* sinv, T rho0, T ih1, T ih2)
{
#pragma unroll
    for (int a = 0; a < kQ; ++a) R.f[a] = Store<S>::dec(R.raw[a], sinv[cls_(a)]);
    const T* f = R.f;
    const T m00 = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const T m10 = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
    const T m01 = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
    R.Fp1 = T(R.Fr[0]);
    R.Fp2 = T(R.Fr[1]);
    R.dr = m00 * ih1 * ih2;
    const T irho = recip_sum(rho0, R.dr);
    R.U1 = (m10 + T(0.5) * R.Fp1) * ih2 * irho;
    R.U2 = (m01 + T(0.5) * R.Fp2) * ih1 * irho;
}

// Work-group -> (strip, segment) of its run.  The hardware deals
// consecutive work-groups to the eight XCDs in turn; the tiles are renumbered
// so that each XCD gets a contiguous band (segment-major), whose halo rows
// and columns its L2 then shares.
__device__ inline void tile_of(const RunDesc& d, int local, int& strip, int& seg)
{
    const int B = d.strips * d.segs;
    const int x = local & 7, idx = local >> 3;
    const int q = B >> 3, rem = B & 7;
    const int t = x * q + min(x, rem) + idx;
    seg = t / d.strips;
    strip = t - seg * d.strips;
}

// One time step for every run of the launch.
//   grid.x = total work-groups, block = 64 (one wave).
//   block_run[b]: run of work-group b.
//   step_ctr[0] + k: the step's index in the sequence of rounding draws.
// A wave owns 62 columns (lanes 1..62; lanes 0 and 63 are the x-halo) and a
// segment of rows, and marches up the rows with three row slots (rows j-1,
// j, j+1); the loads of row j+2 are in flight while row j is collided.
template <class S, bool MHD>
__global__ void __launch_bounds__(kWave) step_kernel(const RunDesc* __restrict__ runs,
                                                     const int32_t* __restrict__ block_run,
                                                     Pools<S, typename ForceOf<S>::type> pl,
                                                     const uint32_t* __restrict__ step_ctr, int k)
{
    using T = typename ComputeOf<S>::type;
    using FT = typename ForceOf<S>::type;
    using Slot = RowSlot<S, T, FT>;
    const int run = block_run[blockIdx.x];
    const RunDesc& d = runs[run];
    int strip, seg;
    tile_of(d, blockIdx.x - d.first_block, strip, seg);
    const int lane = threadIdx.x;
    const NodeParams<T> p0 = node_params<T>(d);
    const uint32_t seed = mix32(step_ctr[0] + uint32_t(k));
    const bool mhd_run = MHD && d.mhd;   // a batch may mix MHD and plain runs

    // lane geometry and column metric
    const int lb = lane_base(d.nx, d.bc_x, strip);
    const int craw = lb + lane;
    const LaneCol L = lane_col(d, craw);
    LaneCol Ls = L;   // the same with in-grid columns for the loads of lanes beyond an x-wall
    if (!L.valid) {
        Ls.col = min(max(craw, 0), d.nx - 1);
        Ls.cm = Ls.cp = Ls.col;
        Ls.wm = Ls.wp = false;
    }
    const int x0 = strip * kOwn;
    const int x1 = min(x0 + kOwn, d.nx);
    const bool own = lane >= 1 && lane <= kWave - 2 && craw >= x0 && craw < x1;
    const bool xwall_lo = d.bc_x != 0 && L.col == 0;
    const bool xwall_hi = d.bc_x != 0 && L.col == d.nx - 1;
    const T* ctab = table_of<T>(pl.col, pl.colf) + (int64_t)(d.col_off + Ls.col) * kTab;
    const T* rtab = table_of<T>(pl.row, pl.rowf) + (int64_t)d.row_off * kTab;
    const T h1_0 = ctab[T_H], ih1_0 = ctab[T_IH], th11_0 = ctab[T_TH];
    const T a1p_0 = ctab[T_AP], a1m_0 = ctab[T_AM], b1p_0 = ctab[T_BP], b1m_0 = ctab[T_BM];
    // per-lane pull offsets of interior rows, relative to the (plane a,
    // row r - ey) base: the source column, or through an x-wall the lane's
    // own node in the opposite plane
    int32_t off[kQ];
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        const int ex = ex_(a), ey = ey_(a);
        if (ex == 0) {
            off[a] = Ls.col;
        } else {
            const bool wx = ex > 0 ? Ls.wm : Ls.wp;
            off[a] = wx ? (opp_(a) - a) * (int32_t)d.plane + ey * d.pitch + Ls.col : (ex > 0 ? Ls.cm : Ls.cp);
        }
    }
    const T* sp = step_params<T>(d);
    T sinv[4], sfw[4], sginv = T(1), sgw = T(1);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        sinv[c] = Store<S>::scaled ? sp[P_ISC + c] : T(1);
        sfw[c] = Store<S>::scaled ? sp[P_SC + c] : T(1);
    }
    if (Store<S>::scaled) {
        sginv = sp[P_ISCG];
        sgw = sp[P_SCG];
    }
    auto ih2_of = [&](int r) { return rtab[(int64_t)r * kTab + T_IH]; };

    int y0, y1;
    seg_rows(d.ny, d.segs, seg, y0, y1);

    // window: A = row y0 - 1, B = row y0, C = row y0 + 1 (loads in flight)
    Slot A, B, C;
    A.dr = A.U2 = T(0);
    if (row_ok(d, y0 - 1)) {
        const int r = row_wrap(d, y0 - 1);
        issue_row<S, FT>(d, pl.fin, pl.Fin, Ls, off, r, A.raw, A.Fr);
        decode_row<S, T, FT>(A, sinv, p0.rho0, ih1_0, ih2_of(r));
    }
    issue_row<S, FT>(d, pl.fin, pl.Fin, Ls, off, y0, B.raw, B.Fr);
    if (mhd_run) issue_row_g<S>(d, pl.gin, Ls, off, y0, B.graw);
    if (row_ok(d, y0 + 1)) issue_row<S, FT>(d, pl.fin, pl.Fin, Ls, off, row_wrap(d, y0 + 1), C.raw, C.Fr);
    decode_row<S, T, FT>(B, sinv, p0.rho0, ih1_0, ih2_of(y0));

    const int64_t plane = d.plane;
    // one row: P = row j - 1, Cs = row j, N = row j + 1
    auto row_step = [&](Slot& P, Slot& Cs, Slot& N, int j) {
        // the scheduler keeps each row to itself (interleaving the unrolled
        // rows only lengthens live ranges); the loads issued here complete
        // during the row's arithmetic
        __builtin_amdgcn_sched_barrier(0);
        // per-row opaque copies of the lane constants
        const NodeParams<T>& p = p0;
        T h1 = h1_0, ih1 = ih1_0, th11 = th11_0, a1p = a1p_0, a1m = a1m_0, b1p = b1p_0, b1m = b1m_0;
        opaque_v(h1);
        opaque_v(ih1);
        opaque_v(th11);
        opaque_v(a1p);
        opaque_v(a1m);
        opaque_v(b1p);
        opaque_v(b1m);
        // 1. loads of row j + 2 (into P, whose populations are done)
        const bool have_next = row_ok(d, j + 1);
        const bool load2 = j + 2 <= y1 && row_ok(d, j + 2);
        if (load2) issue_row<S, FT>(d, pl.fin, pl.Fin, Ls, off, row_wrap(d, j + 2), P.raw, P.Fr);
        // 2. moments of row j + 1
        if (have_next) decode_row<S, T, FT>(N, sinv, p.rho0, ih1, ih2_of(row_wrap(d, j + 1)));

        NodeMetric<T> g;
        g.h1 = h1;
        g.ih1 = ih1;
        g.th11 = th11;
        const T* rt = rtab + (int64_t)j * kTab;
        g.h2 = rt[T_H];
        g.ih2 = rt[T_IH];
        g.th22 = rt[T_TH];
        // 3. differences along xi2 (one-sided next to walls)
        T d2U2, d2r;
        if (d.bc_y != 0 && j == 0) {
            Slot W;
            issue_row<S, FT>(d, pl.fin, pl.Fin, Ls, off, 2, W.raw, W.Fr);
            decode_row<S, T, FT>(W, sinv, p.rho0, ih1, ih2_of(2));
            d2U2 = T(0.5) * (T(-3) * Cs.U2 + T(4) * N.U2 - W.U2);
            d2r = T(0.5) * (T(-3) * Cs.dr + T(4) * N.dr - W.dr);
        } else if (d.bc_y != 0 && j == d.ny - 1) {
            Slot W;
            issue_row<S, FT>(d, pl.fin, pl.Fin, Ls, off, j - 2, W.raw, W.Fr);
            decode_row<S, T, FT>(W, sinv, p.rho0, ih1, ih2_of(j - 2));
            d2U2 = T(0.5) * (T(3) * Cs.U2 - T(4) * P.U2 + W.U2);
            d2r = T(0.5) * (T(3) * Cs.dr - T(4) * P.dr + W.dr);
        } else {
            d2U2 = T(0.5) * (N.U2 - P.U2);
            d2r = T(0.5) * (N.dr - P.dr);
        }
        // differences along xi1 from the neighbouring lanes
        const T drho = Cs.dr, rho = p.rho0 + drho, U1 = Cs.U1, U2 = Cs.U2;
        // (the lane shifts run with every lane active: a shift inside a
        // lane-divergent branch would read inactive lanes)
        const T Um1 = from_prev(U1), Up1 = from_next(U1);
        const T rm1 = from_prev(drho), rp1 = from_next(drho);
        T d1U1 = T(0.5) * (Up1 - Um1), d1r = T(0.5) * (rp1 - rm1);
        if (d.bc_x != 0) {   // one-sided next to x-walls
            const T Up2 = from_next(Up1), rp2 = from_next(rp1);
            const T Um2 = from_prev(Um1), rm2 = from_prev(rm1);
            if (xwall_lo) {
                d1U1 = T(0.5) * (T(-3) * U1 + T(4) * Up1 - Up2);
                d1r = T(0.5) * (T(-3) * drho + T(4) * rp1 - rp2);
            } else if (xwall_hi) {
                d1U1 = T(0.5) * (T(3) * U1 - T(4) * Um1 + Um2);
                d1r = T(0.5) * (T(3) * drho - T(4) * rm1 + rm2);
            }
        }

        // 4. App. G: magnetic field, local derivatives, Lorentz force,
        //    collision and the D2Q5 writes (stored value = base + increment;
        //    anti-bounce-back slots negate the post-collision value); then the
        //    D2Q5 loads of row j + 1, in flight during the fluid collision
        T Fx1 = p.Fx1, Fx2 = p.Fx2;
        const RowGeo Gj = row_geo(d, j);
        const int64_t nn = (int64_t)j * d.pitch + L.col;
        const uint32_t hn = mix32(uint32_t(d.f_off + nn) ^ seed);
        if (mhd_run) {
            T dg[2][kM], dgi[2][kM];
#pragma unroll
            for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                for (int a = 0; a < kM; ++a) dg[ci][a] = T(Store<S>::dec(Cs.graw[ci][a], sginv));
            T B1, B2, FL1, FL2;
            mie_node<T>(p, g, dg, U1, U2, B1, B2, FL1, FL2, dgi);
            Fx1 += FL1;
            Fx2 += FL2;
            if (own) {
                const T b2p = rt[T_BP], b2m = rt[T_BM];
                const T hh = g.h1 * g.h2;
#pragma unroll
                for (int a = 1; a < kM; ++a) {
                    const int ex = ex_(a), ey = ey_(a);
                    const bool wx = (ex > 0 && L.wp) || (ex < 0 && L.wm);
                    const bool wy = (ey > 0 && Gj.wp) || (ey < 0 && Gj.wm);
                    if (wx || wy) {
                        // anti-bounce-back of App. G: the reader (this node) sees
                        // -g~ + 2 W h_wall B_wall with B_wall = (0, B0)
                        const T hwall = wy ? g.h1 * sp[ey < 0 ? P_HWLO : P_HWHI]
                                           : sp[ex < 0 ? P_H1WLO : P_H1WHI] * g.h2;
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
            if (j + 1 < y1) issue_row_g<S>(d, pl.gin, Ls, off, row_wrap(d, j + 1), N.graw);
        }

        // 5. effective force, corrections, central-moment collision
        T F1, F2, n3, n4, inc[kQ];
        force_and_corrections<T>(p, g, rho, drho, U1, U2, d1U1, d2U2, d1r, d2r, Fx1, Fx2, F1, F2, n3, n4);
        cm_collide<T>(p, g, raw_dev<T>(Cs.f), rho, drho, U1, U2, Cs.Fp1, Cs.Fp2, F1, F2, n3, n4, inc);

        // 6. D2Q9 writes: inc holds the collision increments; the writer adds the
        //    rest-state offsets of the interior axis slots (the reader is the
        //    neighbour; its rest state differs through the metric) and the
        //    reader's wall terms
        if (own) {
            const T a2p = rt[T_AP], a2m = rt[T_AM];
            inc[1] += g.h2 * a1p;
            inc[3] += g.h2 * a1m;
            inc[2] += g.h1 * a2p;
            inc[4] += g.h1 * a2m;
            // momentum-augmented bounce-back of App. C for populations
            // leaving through a moving y-wall
            if (Gj.wp && d.uw_hi != 0.0) {
                const T cw = rho * sp[P_CWHI];
                // slot 5 is read back as f7, slot 6 as f8: f7 = ft5 - cw, f8 = ft6 + cw
                if (d.lid_corners || !xwall_hi) inc[5] -= cw;
                if (d.lid_corners || !xwall_lo) inc[6] += cw;
            }
            if (Gj.wm && d.uw_lo != 0.0) {
                const T cw = rho * sp[P_CWLO];
                // slot 7 is read back as f5, slot 8 as f6: f5 = ft7 + cw, f6 = ft8 - cw
                if (d.lid_corners || !xwall_lo) inc[7] += cw;
                if (d.lid_corners || !xwall_hi) inc[8] -= cw;
            }
            S* fo = pl.fout + d.f_off + nn;
#pragma unroll
            for (int a = 0; a < kQ; ++a)
                Store<S>::st_sr(fo, a * plane, Cs.f[a], inc[a], sfw[cls_(a)], pop_draw(hn, a));
            pl.Fout[d.F_off + nn] = FT(F1);
            pl.Fout[d.F_off + nn + plane] = FT(F2);
        }
        __builtin_amdgcn_sched_barrier(0);
    };

    // march with the three slots rotating roles (no moves between rows)
    for (int j = y0; j < y1; j += 3) {
        row_step(A, B, C, j);
        if (j + 1 >= y1) break;
        row_step(B, C, A, j + 1);
        if (j + 2 >= y1) break;
        row_step(C, A, B, j + 2);
    }
}

}  // namespace goc
