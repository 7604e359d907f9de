// goc_curv.hpp -- the time step on a general orthogonal grid.
//
// A run whose metric factors vary with both coordinates (h1(xi1, xi2),
// h2(xi1, xi2); theta12, theta21 != 0: curvilinear body-fitted grids such as
// the conformal annular sector) keeps the slot layout, the deviation
// storage and the writer-side boundary conditions of the straight path, with
// the metric read per node from a pool of planes (goc_device.hpp: M_*).  A
// step is one launch of one thread per node over 64 x 8 tiles: pull, decode
// and the moments rho - rho0, U1, U2 (App. E step 7, lagged force) of the
// tile and of the ring of nodes around it into LDS; the second-order
// differences of U and rho from LDS (one-sided next to walls, wrapped when
// periodic); the general stresses and effective force with the local shear
// stress (Sec. 2.2, App. A), the corrections of Sec. 5 with their curvature
// terms, the collision, and the writes of the nine slots, their ghost-row
// copies and the force.  The ring is pulled twice (by this tile and by its
// owner), which costs L2 reads, not HBM traffic.  The D2Q5 induction scheme
// is not part of this path (the library refuses MHD runs on 2-D metrics).
#pragma once

#include "goc_step.hpp"

namespace goc {

constexpr int kCurvX = 64, kCurvY = 8;   // work-group tile: 64 columns x 8 rows

// Metric of node n of a 2-D run in the compute type.
template <class T, class S, class FT>
__device__ inline NodeMetric<T> curv_metric(const RunDesc& d, const Pools<S, FT>& pl, int64_t n, int64_t N,
                                            T& aE, T& aW, T& aN, T& aS)
{
    const T* m = table_of<T>(pl.met, pl.metf) + d.met_off + n;
    NodeMetric<T> g;
    g.h1 = m[M_H1 * N];
    g.ih1 = m[M_IH1 * N];
    g.h2 = m[M_H2 * N];
    g.ih2 = m[M_IH2 * N];
    g.th11 = m[M_TH11 * N];
    g.th12 = m[M_TH12 * N];
    g.th21 = m[M_TH21 * N];
    g.th22 = m[M_TH22 * N];
    aE = m[M_AE * N];
    aW = m[M_AW * N];
    aN = m[M_AN * N];
    aS = m[M_AS * N];
    return g;
}

// Element offset, from row 0 of a slot region, of the slot node (i, j)
// pulls for direction a: through an xi1-wall its own slot of the opposite
// direction; otherwise slot a of the source node x - e_a, wrapped across a
// periodic xi1, in rows -1 .. ny (the ghost rows hold what lies beyond the
// domain in xi2).  The same gather as the straight march.
__device__ inline int64_t curv_pull(const RunDesc& d, int i, int j, int a)
{
    const int ex = ex_(a), ey = ey_(a);
    int si = i - ex;
    if (si < 0 || si >= d.nx) {
        if (d.bc_x != 0) return (int64_t)opp_(a) * d.plane + (int64_t)j * d.pitch + i;
        si = si < 0 ? si + d.nx : si - d.nx;
    }
    return (int64_t)a * d.plane + (int64_t)(j - ey) * d.pitch + si;
}

// Pull and decode the nine deviations of node (i, j) and its lagged force.
template <class S, class T, class FT>
__device__ inline void curv_pull9(const RunDesc& d, const Pools<S, FT>& pl, int i, int j, T* f, T& Fp1, T& Fp2)
{
    const T* sp = step_params<T>(d);
    const S* base = pl.fin + d.f_off;
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        const T sinv = Store<S>::scaled ? sp[P_ISC + cls_(a)] : T(1);
        f[a] = T(Store<S>::ld(base, curv_pull(d, i, j, a), sinv));
    }
    const int64_t nf = d.F_off + (int64_t)j * d.pitchF + i;
    Fp1 = T(pl.Fin[nf]);
    Fp2 = T(pl.Fin[nf + d.plane]);
}

// Moments of a pulled node, as the straight march forms them: dr = rho -
// rho0 = dm00/(h1 h2), U1 = (dm10 + F1/2)/(rho h2), U2 = (dm01 + F2/2)/(rho h1).
template <class T>
__device__ inline void curv_moments(const T* f, T Fp1, T Fp2, T rho0, T ih1, T ih2, T& dr, T& U1, T& U2)
{
    const T m00 = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const T m10 = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
    const T m01 = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
    dr = m00 * ih1 * ih2;
    const T irho = recip_sum(rho0, dr);
    U1 = (m10 + T(0.5) * Fp1) * ih2 * irho;
    U2 = (m01 + T(0.5) * Fp2) * ih1 * irho;
}

// Second-order difference along one axis of a node field held in a tile:
// central inside and across a periodic edge (the halo holds the wrapped
// neighbours), one-sided (-3 p0 + 4 p1 - p2)/2 next to a wall.  v(l) reads
// the tile at local index l; k is the node's index on the axis, n its length.
template <class T, class V>
__device__ inline T tile_fd(V v, int l, int k, int n, bool periodic)
{
    if (!periodic && k == 0) return T(0.5) * (T(-3) * v(l) + T(4) * v(l + 1) - v(l + 2));
    if (!periodic && k == n - 1) return T(0.5) * (T(3) * v(l) - T(4) * v(l - 1) + v(l - 2));
    return T(0.5) * (v(l + 1) - v(l - 1));
}

// The step of every node of one run.  Launch: grid (ceil(nx/64),
// ceil(ny/8)), block (64, 8).  A work-group owns the 64 x 8 nodes at
// (64 bx, 8 by); its tile is shifted back at the far edges of the grid so
// that the three nodes of a one-sided difference lie in it (nodes of the
// shifted part belong to the neighbouring work-group and are not written
// here).  The moments of the tile and of the ring around it go to LDS.
template <class S, int COLL>
__global__ void __launch_bounds__(kCurvX * kCurvY)
curv_step_kernel(const RunDesc* __restrict__ runs, int run, Pools<S, typename ForceOf<S>::type> pl,
                 const uint32_t* __restrict__ step_ctr, int k)
{
    using T = typename ComputeOf<S>::type;
    using FT = typename ForceOf<S>::type;
    __shared__ T sm[3][kCurvY + 2][kCurvX + 2];   // rho - rho0, U1, U2 of the tile and its ring
    const RunDesc& d = runs[run];
    const int nx = d.nx, ny = d.ny;
    const int tx = nx < kCurvX ? nx : kCurvX, ty = ny < kCurvY ? ny : kCurvY;   // tile extent
    const int ox = blockIdx.x * kCurvX, oy = blockIdx.y * kCurvY;              // first owned node
    const int x0 = ox < nx - tx ? ox : nx - tx, y0 = oy < ny - ty ? oy : ny - ty;   // tile origin
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int i = x0 + lx, j = y0 + ly;
    const bool in = lx < tx && ly < ty;
    const bool px = d.bc_x == 0, py = d.bc_y == 0;
    const int64_t N = (int64_t)nx * ny, n = (int64_t)j * nx + i;
    const NodeParams<T> p = node_params<T>(d);
    const T* sp = step_params<T>(d);
    NodeMetric<T> g{};
    T aE = 0, aW = 0, aN = 0, aS = 0, f[kQ] = {}, Fp1 = 0, Fp2 = 0, dr = 0, U1 = 0, U2 = 0;
    if (in) {
        g = curv_metric<T>(d, pl, n, N, aE, aW, aN, aS);
        curv_pull9<S, T, FT>(d, pl, i, j, f, Fp1, Fp2);
        curv_moments<T>(f, Fp1, Fp2, p.rho0, g.ih1, g.ih2, dr, U1, U2);
        sm[0][ly + 1][lx + 1] = dr;
        sm[1][ly + 1][lx + 1] = U1;
        sm[2][ly + 1][lx + 1] = U2;
    }
    // the ring: rows -1 and ty over the tile's columns, columns -1 and tx over
    // its rows (the differences never reach the corners); wrapped across a
    // periodic edge, absent beyond a wall
    const T* mt = table_of<T>(pl.met, pl.metf) + d.met_off;
    const int nh = 2 * tx + 2 * ty;
    for (int h = ly * kCurvX + lx; h < nh; h += kCurvX * kCurvY) {
        int hx, hy;
        if (h < 2 * tx) {
            hx = h < tx ? h : h - tx;
            hy = h < tx ? -1 : ty;
        } else {
            hx = h < 2 * tx + ty ? -1 : tx;
            hy = h < 2 * tx + ty ? h - 2 * tx : h - 2 * tx - ty;
        }
        int hi = x0 + hx, hj = y0 + hy;
        if (hi < 0 || hi >= nx) {
            if (!px) continue;
            hi = hi < 0 ? hi + nx : hi - nx;
        }
        if (hj < 0 || hj >= ny) {
            if (!py) continue;
            hj = hj < 0 ? hj + ny : hj - ny;
        }
        const int64_t hn = (int64_t)hj * nx + hi;
        T hf[kQ], hF1, hF2, hdr, hU1, hU2;
        curv_pull9<S, T, FT>(d, pl, hi, hj, hf, hF1, hF2);
        curv_moments<T>(hf, hF1, hF2, p.rho0, mt[M_IH1 * N + hn], mt[M_IH2 * N + hn], hdr, hU1, hU2);
        sm[0][hy + 1][hx + 1] = hdr;
        sm[1][hy + 1][hx + 1] = hU1;
        sm[2][hy + 1][hx + 1] = hU2;
    }
    __syncthreads();
    if (!in || i < ox || j < oy) return;

    const T rho = p.rho0 + dr;
    const int cx = lx + 1, cy = ly + 1;
    const T d1U1 = tile_fd<T>([&](int c) { return sm[1][cy][c]; }, cx, i, nx, px);
    const T d1r = tile_fd<T>([&](int c) { return sm[0][cy][c]; }, cx, i, nx, px);
    const T d2U2 = tile_fd<T>([&](int r) { return sm[2][r][cx]; }, cy, j, ny, py);
    const T d2r = tile_fd<T>([&](int r) { return sm[0][r][cx]; }, cy, j, ny, py);

    const RawDev<T> m = raw_dev<T>(f);
    T F1, F2, n3, n4, inc[kQ];
    force_and_corrections_gen<T>(p, g, rho, dr, U1, U2, d1U1, d2U2, d1r, d2r, p.Fx1, p.Fx2, m.m11, F1, F2, n3,
                                 n4);
    if constexpr (COLL == kCollRaw)
        raw_collide<T>(p, g, m, rho, dr, U1, U2, Fp1, Fp2, F1, F2, n3, n4, inc);
    else
        cm_collide<T>(p, g, m, rho, dr, U1, U2, Fp1, Fp2, F1, F2, n3, n4, inc);

    // writer side: rest-state offsets of the axis slots (their readers are the
    // neighbours; zero toward walls) and the wall terms of App. C
    inc[1] += aE;
    inc[3] += aW;
    inc[2] += aN;
    inc[4] += aS;
    const bool wxlo = !px && i == 0, wxhi = !px && i == nx - 1;
    const bool wylo = !py && j == 0, wyhi = !py && j == ny - 1;
    const double* face = pl.face + d.face_off;   // [2 ny] h1 on the xi1 faces, then [2 nx] h2 on the xi2 faces
    if (wyhi && d.uw_hi != 0.0) {
        const T cw = rho * T(0.5) * p.cs2 * T(d.uw_hi) / T(face[2 * ny + 2 * i + 1]);
        if (d.lid_corners || !wxhi) inc[5] -= cw;
        if (d.lid_corners || !wxlo) inc[6] += cw;
    }
    if (wylo && d.uw_lo != 0.0) {
        const T cw = rho * T(0.5) * p.cs2 * T(d.uw_lo) / T(face[2 * ny + 2 * i]);
        if (d.lid_corners || !wxlo) inc[7] += cw;
        if (d.lid_corners || !wxhi) inc[8] -= cw;
    }
    if (wxhi && d.vw_hi != 0.0) {
        const T cx = rho * T(0.5) * p.cs2 * T(d.vw_hi) / T(face[2 * j + 1]);
        if (d.lid_corners || !wyhi) inc[5] -= cx;
        if (d.lid_corners || !wylo) inc[8] += cx;
    }
    if (wxlo && d.vw_lo != 0.0) {
        const T cx = rho * T(0.5) * p.cs2 * T(d.vw_lo) / T(face[2 * j]);
        if (d.lid_corners || !wylo) inc[7] += cx;
        if (d.lid_corners || !wyhi) inc[6] -= cx;
    }

    // stores: base + increment, rounded without bias (the same draws as the
    // straight march: node, population, step)
    const uint32_t seed = mix32(step_ctr[0] + uint32_t(k));
    const int64_t nn = (int64_t)j * d.pitch + i;
    const uint32_t hn = mix32(uint32_t(d.f_off + nn) ^ seed);
    S* out = pl.fout + d.f_off;
    S e[kQ];
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        const T sfw = Store<S>::scaled ? sp[P_SC + cls_(a)] : T(1);
        e[a] = Store<S>::enc(f[a], inc[a], sfw, pop_draw(hn, a));
        out[(int64_t)a * d.plane + nn] = e[a];
    }
    // ghost rows (rows 0 and ny - 1): walls take the bounced values at the
    // reader's source column, into the row beyond the wall; periodic xi2 takes
    // copies of the slots the opposite edge row pulls, into the ghost row
    // beyond that edge.  Planes: walls bottom {2, 5, 6}, top {4, 8, 7};
    // periodic bottom {4, 7, 8}, top {2, 6, 5}.
    const bool bot = j == 0, top = j == ny - 1;
    if (bot || top) {
        const bool wall = !py;
        const int grow = (wall ? bot : top) ? -1 : ny;
        const int p0 = (wall == bot) ? 2 : 4;
        const int p1 = wall ? (bot ? 5 : 8) : (bot ? 7 : 6);
        const int p2 = wall ? (bot ? 6 : 7) : (bot ? 8 : 5);
        const int cm = px ? (i == 0 ? nx - 1 : i - 1) : i - 1;
        const int cp = px ? (i == nx - 1 ? 0 : i + 1) : i + 1;
        S* gr = out + (int64_t)grow * d.pitch;
        gr[(int64_t)p0 * d.plane + i] = bot ? e[4] : e[2];
        if (!wall) {
            gr[(int64_t)p1 * d.plane + i] = bot ? e[7] : e[6];
            gr[(int64_t)p2 * d.plane + i] = bot ? e[8] : e[5];
        } else {
            if (!wxlo) gr[(int64_t)p1 * d.plane + cm] = bot ? e[7] : e[6];
            if (!wxhi) gr[(int64_t)p2 * d.plane + cp] = bot ? e[8] : e[5];
        }
    }
    const int64_t nf = d.F_off + (int64_t)j * d.pitchF + i;
    pl.Fout[nf] = FT(F1);
    pl.Fout[nf + d.plane] = FT(F2);
}

}  // namespace goc
