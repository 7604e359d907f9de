// goc_tile.hpp -- the tiled time step: one thread per node over LDS tiles.
//
// The same step as the march of goc_step.hpp (App. E, every node once),
// organised for parallelism instead of in-register reuse: a work-group owns
// a tile of 64 columns x 4, 8 or 16 rows, or 128 x 4, and steps it in one
// pass.  Pull,
// decode and the moments rho - rho0, U1, U2 (App. E step 7, lagged force)
// of the tile and of the ring of nodes around it go to LDS; after one
// barrier the second-order differences of U and rho come from LDS
// (one-sided next to walls, wrapped when periodic); then the stresses and
// effective force (Sec. 2.2, App. A), the corrections of Sec. 4, the
// collision and the writes of the nine slots, their ghost-row copies and
// the force.  The ring is pulled twice (by this tile and by its owner),
// which costs L2 reads, not HBM traffic.  Two metric sources:
//  - GEN: a run whose metric factors vary with both coordinates (h1(xi1,
//    xi2), h2(xi1, xi2); theta12, theta21 != 0: curvilinear body-fitted
//    grids such as the conformal annular sector) reads its metric per node
//    from a pool of planes (goc_device.hpp: M_*), with the general stresses,
//    the local shear stress and the curvature terms of the corrections;
//  - otherwise the column and row tables of a straight grid and the march's
//    arithmetic, including (MHD) the D2Q5 scheme of App. G, whose node work
//    is local.  The D2Q5 scheme does not run on 2-D metrics (the library
//    refuses MHD runs there).
#pragma once

#include "goc_step.hpp"

namespace goc {

constexpr int kTileX = 64;   // work-group tile: 64 columns x TY rows (one wave per row)
// Tile heights the library instantiates (the autotuner picks one per handle)
// and the default: 8 rows, 4 for FP64 storage, whose register count leaves
// room for fewer waves per CU.
constexpr int kTileRows[3] = {4, 8, 16};
// The wide tile: 128 columns (two waves per row of the tile) at 4 rows.  Its
// longer row pieces suit the memory system on wide grids larger than the
// caches; its ring per node is that of the 64 x 4 tile.
constexpr int kTileXWide = 128;
constexpr int kTileRowsWide = 4;
constexpr int default_tile_rows(int storage_bytes) { return storage_bytes == 8 ? 4 : 8; }

// A value at a lane's 32-bit byte offset from a work-group-uniform base:
// the hardware forms such an address from a scalar base and a vector
// offset, with no 64-bit arithmetic per lane.  Every offset of a run lies
// below 4 GiB (the library refuses larger runs at creation).
template <class V>
__device__ inline V ld_at(const void* base, uint32_t off)
{
    return *reinterpret_cast<const V*>(static_cast<const char*>(base) + off);
}
template <class V>
__device__ inline void st_at(void* base, uint32_t off, V v)
{
    *reinterpret_cast<V*>(static_cast<char*>(base) + off) = v;
}
// The same as a non-temporal store when NT: where the state is larger than
// the caches, the step's outputs are read once, by the next step, after the
// whole state has streamed through them, so keeping them cached only
// displaces the data in flight (measured on the step's access pattern
// without arithmetic, 4096 x 1024 with the D2Q5 slots: 142.6 us per launch
// with plain stores, 134.5 us non-temporal); where it fits in the Infinity
// Cache, the next step reads it from there, and plain stores keep it.
template <bool NT, class V>
__device__ inline void st_nt(void* base, uint32_t off, V v)
{
    char* p = static_cast<char*>(base) + off;
    if constexpr (!NT)
        *reinterpret_cast<V*>(p) = v;
    else if constexpr (sizeof(V) == 2)
        __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), reinterpret_cast<uint16_t*>(p));
    else if constexpr (sizeof(V) == 4)
        __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, v), reinterpret_cast<uint32_t*>(p));
    else
        __builtin_nontemporal_store(__builtin_bit_cast(uint64_t, v), reinterpret_cast<uint64_t*>(p));
}

// Metric of a node of a 2-D run in the compute type: nb = its node index
// times sizeof(T), NB = one plane of the run in bytes.
template <class T, class S, class FT>
__device__ inline NodeMetric<T> tile_metric2d(const RunDesc& d, const Pools<S, FT>& pl, uint32_t nb, int64_t NB,
                                            T& aE, T& aW, T& aN, T& aS)
{
    const char* m = reinterpret_cast<const char*>(table_of<T>(pl.met, pl.metf) + d.met_off);
    NodeMetric<T> g;
    g.h1 = ld_at<T>(m + M_H1 * NB, nb);
    g.ih1 = ld_at<T>(m + M_IH1 * NB, nb);
    g.h2 = ld_at<T>(m + M_H2 * NB, nb);
    g.ih2 = ld_at<T>(m + M_IH2 * NB, nb);
    g.th11 = ld_at<T>(m + M_TH11 * NB, nb);
    g.th12 = ld_at<T>(m + M_TH12 * NB, nb);
    g.th21 = ld_at<T>(m + M_TH21 * NB, nb);
    g.th22 = ld_at<T>(m + M_TH22 * NB, nb);
    aE = ld_at<T>(m + M_AE * NB, nb);
    aW = ld_at<T>(m + M_AW * NB, nb);
    aN = ld_at<T>(m + M_AN * NB, nb);
    aS = ld_at<T>(m + M_AS * NB, nb);
    return g;
}

// Byte offset of the slot node (i, j) pulls for direction a, from the base
// of a slot region (ghost row -1), as in the straight march: slot a of the
// source node x - e_a, wrapped across a periodic xi1, in rows -1 .. ny (the
// ghost rows hold what lies beyond the domain in xi2); through an xi1-wall
// the node's own slot of the opposite direction.  The node's own offset plus
// a work-group-uniform constant per direction, selected per lane at the xi1
// edges.  The D2Q5 slots (a < 5) are pulled the same way, within their
// component's five planes.
template <class S>
__device__ inline uint32_t pull_off(const RunDesc& d, const RunBytes& b, int i, int j, int a)
{
    const uint32_t cs = uint32_t(sizeof(S));
    const uint32_t o = uint32_t(j + 1) * b.pitch_s + uint32_t(i) * cs;   // own node, plane 0
    const int ex = ex_(a), ey = ey_(a);
    uint32_t off = o + uint32_t(a) * b.plane_s - uint32_t(ey) * b.pitch_s - uint32_t(ex) * cs;
    if (ex != 0) {
        const bool out = ex > 0 ? i == 0 : i == d.nx - 1;
        const uint32_t span = uint32_t(d.nx) * cs;
        const uint32_t wrapped = ex > 0 ? off + span : off - span;
        const uint32_t bounced = o + uint32_t(opp_(a)) * b.plane_s;
        off = out ? (d.bc_x != 0 ? bounced : wrapped) : off;
    }
    return off;
}

// Pull and decode the nine deviations of node (i, j) and its lagged force
// (planeF: one force plane in bytes).  16-bit storage: ref = the reference
// entries of the node's row (the deviation is stored minus them).
template <class S, class T, class FT, class R>
__device__ inline void tile_pull9(const RunDesc& d, const RunBytes& b, uint32_t planeF, int i, int j, R ref,
                                  T* f, T& Fp1, T& Fp2)
{
    const T* sp = step_params<T>(d);
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        if constexpr (Store<S>::scaled)
            f[a] = Store<S>::dec(ld_at<S>(b.f, pull_off<S>(d, b, i, j, a)), sp[P_ISC + cls_(a)]) + ref[a];
        else
            f[a] = T(Store<S>::dec(ld_at<S>(b.f, pull_off<S>(d, b, i, j, a)), T(1)));
    }
    const uint32_t nf = uint32_t(j) * b.pitch_F + uint32_t(i) * uint32_t(sizeof(FT));
    Fp1 = T(ld_at<FT>(b.F, nf));
    Fp2 = T(ld_at<FT>(b.F, nf + planeF));
}

// Pull and decode the ten D2Q5 deviations of node (i, j) (sginv: the
// inverse storage scale; 16-bit storage: ref as for tile_pull9).
template <class S, class T, class R>
__device__ inline void pull_g(const RunDesc& d, const RunBytes& b, int i, int j, T sginv, R ref, T (*dg)[kM])
{
#pragma unroll
    for (int a = 0; a < kM; ++a) {
        const uint32_t off = pull_off<S>(d, b, i, j, a);
#pragma unroll
        for (int ci = 0; ci < 2; ++ci) {
            dg[ci][a] = T(Store<S>::dec(ld_at<S>(b.g, ci * b.g_comp + off), sginv));
            if constexpr (Store<S>::scaled) dg[ci][a] += ref[kRefG + ci * kM + a];
        }
    }
}

// Reference of the reader of each slot a node writes (16-bit storage): the
// reader's row and direction, i.e. row j + e_a2 (wrapped when periodic) and
// direction a, or, where the slot leaves through a y-wall, the node itself in
// row j with the opposite direction.  R0, Rm, Rp: the entries of rows j,
// j - 1 and j + 1 (first: the entry of direction 0), wylo / wyhi: the node's
// row lies next to a y-wall; all uniform over a wave (one row per wave), so
// the references are scalar values.  n directions of one D2Q9 or D2Q5 set.
template <int n, class R>
__device__ inline void reader_refs(R R0, R Rm, R Rp, bool wylo, bool wyhi, float* ro)
{
#pragma unroll
    for (int a = 0; a < n; ++a) {
        const int ey = ey_(a);
        const bool bounced = (ey > 0 && wyhi) || (ey < 0 && wylo);
        // (the choice is made on the uniform address, so one scalar load reads it)
        const R src = bounced ? R0 + opp_(a) : ey > 0 ? Rp + a : ey < 0 ? Rm + a : R0 + a;
        ro[a] = *src;
    }
}

// The slots that leave through an xi1-wall are read by the node itself with
// the opposite direction: the change of reference, added to the increments
// of those slots of the nodes beside the wall (n directions as above).
template <int n, class R, class T>
__device__ inline void xwall_refs(R R0, const float* ro, bool wxlo, bool wxhi, T* inc)
{
#pragma unroll
    for (int a = 0; a < n; ++a) {
        const int ex = ex_(a);
        if (ex == 0) continue;
        const bool bounced = (ex > 0 && wxhi) || (ex < 0 && wxlo);
        if (bounced) inc[a] -= T(R0[opp_(a)] - ro[a]);
    }
}

// Moments of a pulled node, as the straight march forms them: dr = rho -
// rho0 = dm00/(h1 h2), U1 = (dm10 + F1/2)/(rho h2), U2 = (dm01 + F2/2)/(rho h1).
template <class T>
__device__ inline void tile_moments(const T* f, T Fp1, T Fp2, T rho0, T ih1, T ih2, T& dr, T& U1, T& U2)
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

// Extent and origin along one axis of n nodes of the tile whose first owned
// node is o (tile size T): the owned part, which is shorter than T at the
// far edge of the axis; only where a wall ends the axis with fewer than
// three nodes left is the tile shifted back to full size instead, so that
// the three nodes of a one-sided difference lie in it (the nodes of the
// shifted part belong to the neighbouring work-group and are not written).
__host__ __device__ inline void tile_span(int n, int T, int o, bool periodic, int& ext, int& org)
{
    const int rest = n - o;
    if (rest >= T || periodic || rest >= 3) {
        ext = rest < T ? rest : T;
        org = o;
    } else {
        ext = n < T ? n : T;
        org = n - ext;
    }
}

// The step of every node of every run.  Launch: grid = the tiles of all
// runs (1-D), block (TX, TY) with TX = 64 or 128 columns; NT: non-temporal
// stores; tile_first[r] = the first tile of run r (tile_first[nruns] = all
// tiles), a run's tiles being ceil(nx/TX) * ceil(ny/TY) in row-major order.
// A work-group owns the TX x TY nodes of tile (bx, by) of its run at
// (TX bx, TY by), fewer at the far edges of the grid (tile_span; the threads
// beyond them load a node of the tile and store nothing).  The moments of
// the tile and of the ring around it go to LDS.  The hardware deals consecutive work-groups to
// the eight XCDs in turn; the tiles are renumbered so that each XCD gets a
// contiguous band of them (run by run, row-major), whose rings and
// cross-tile pulls its L2 then serves.
template <class S, int COLL, bool GEN, bool MHD, int TY, bool NT, int TX = kTileX>
__global__ void __launch_bounds__(TX * TY)
tile_step_kernel(const RunDesc* __restrict__ runs, const int32_t* __restrict__ tile_first, int nruns,
                 Pools<S, typename ForceOf<S>::type> pl, const uint32_t* __restrict__ step_ctr, int k)
{
    using T = typename ComputeOf<S>::type;
    using FT = typename ForceOf<S>::type;
    constexpr int kTileY = TY;
    __shared__ T sm[3][kTileY + 2][TX + 2];   // rho - rho0, U1, U2 of the tile and its ring
    // tile of this work-group over all runs, in XCD bands, then its run (the
    // last whose first tile is not beyond it) and its place in the run
    const int nt = tile_first[nruns];
    const int xcd = blockIdx.x & 7, q = nt >> 3, rem = nt & 7;
    const int tg = xcd * q + min(xcd, rem) + (int)(blockIdx.x >> 3);
    int rlo = 0, rhi = nruns - 1;
    while (rlo < rhi) {
        const int mid = (rlo + rhi + 1) >> 1;
        if (tile_first[mid] <= tg) rlo = mid;
        else rhi = mid - 1;
    }
    const int run = rlo;
    const int t = tg - tile_first[run];
    const RunDesc& d = runs[run];
    const int nx = d.nx, ny = d.ny;
    const int gx = (nx + TX - 1) / TX;
    const int ox = (t % gx) * TX, oy = (t / gx) * kTileY;          // first owned node
    const bool mhd_run = MHD && d.mhd;   // (a plain run of a mixed batch: no D2Q5 work)
    const bool px = d.bc_x == 0, py = d.bc_y == 0;
    int tx, ty, x0, y0;   // tile extent and origin
    tile_span(nx, TX, ox, px, tx, x0);
    tile_span(ny, kTileY, oy, py, ty, y0);
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int i = x0 + lx, j = y0 + ly;
    const bool in = lx < tx && ly < ty;
    const int64_t NB = (int64_t)nx * ny * sizeof(T);   // one metric plane in bytes
    const RunBytes b = run_bytes(d, pl);
    const uint32_t planeF = uint32_t(d.plane * sizeof(FT));
    const NodeParams<T> p = node_params<T>(d);
    const T* sp = step_params<T>(d);
    const char* mt = reinterpret_cast<const char*>(table_of<T>(pl.met, pl.metf) + d.met_off);
    // the own node, clamped into the grid for the threads of a ragged tile
    // that have none (they load, but store nothing); its row, uniform over
    // the wave (each wave lies in one row of the tile: lane 0 holds a node
    // of that row whenever any lane of the wave does, and lanes without a
    // node compute nothing that is kept)
    const int ic = in ? i : x0, jc = in ? j : y0;
    const int jw = __builtin_amdgcn_readfirstlane(jc);
    // this thread's node of the ring around the tile: rows -1 and ty over the
    // tile's columns, columns -1 and tx over its rows (the differences never
    // reach the corners); wrapped across a periodic edge, absent beyond a
    // wall.  Ring node h goes to thread h in order (whole rows of the ring
    // per wave: contiguous loads), and the waves beyond the ring skip it.
    static_assert(2 * TX + 2 * kTileY <= TX * kTileY, "one ring node per thread");
    const int h = ly * TX + lx, nh = 2 * tx + 2 * ty;
    int hx, hy;
    if (h < 2 * tx) {
        hx = h < tx ? h : h - tx;
        hy = h < tx ? -1 : ty;
    } else {
        hx = h < 2 * tx + ty ? -1 : tx;
        hy = h < 2 * tx + ty ? h - 2 * tx : h - 2 * tx - ty;
    }
    int hi = x0 + hx, hj = y0 + hy;
    bool hv = h < nh;
    if (hi < 0 || hi >= nx) {
        hv = hv && px;
        hi = hi < 0 ? hi + nx : hi - nx;
    }
    if (hj < 0 || hj >= ny) {
        hv = hv && py;
        hj = hj < 0 ? hj + ny : hj - ny;
    }
    hi = hv ? hi : ic;
    hj = hv ? hj : jc;
    // the loads of the own node, then (in a wave holding ring nodes) those of
    // the ring node, before either node's moments: one wait for both
    const uint32_t hnb = uint32_t(hj * nx + hi) * uint32_t(sizeof(T));
    // GEN: the metric planes and the writer's rest-state offsets of the four
    // axis slots; otherwise the column and row tables of the straight grid
    // (the offsets a1+-, a2+- are scaled by h2 / h1 at the writes)
    T aE, aW, aN, aS, b1p = 0, b1m = 0, b2p = 0, b2m = 0;
    NodeMetric<T> g;
    const T* ctab = table_of<T>(pl.col, pl.colf) + (int64_t)d.col_off * kTab;
    const T* rtab = table_of<T>(pl.row, pl.rowf) + (int64_t)d.row_off * kTab;
    if constexpr (GEN) {
        g = tile_metric2d<T>(d, pl, uint32_t(jc * nx + ic) * uint32_t(sizeof(T)), NB, aE, aW, aN, aS);
    } else {
        const T* ct = ctab + ic * kTab;
        const CPtr<T> rt = (CPtr<T>)(rtab + jw * kTab);   // (scalar loads)
        g.h1 = ct[T_H];
        g.ih1 = ct[T_IH];
        g.th11 = ct[T_TH];
        g.h2 = rt[T_H];
        g.ih2 = rt[T_IH];
        g.th22 = rt[T_TH];
        g.th12 = g.th21 = T(0);
        aE = ct[T_AP];
        aW = ct[T_AM];
        aN = rt[T_AP];
        aS = rt[T_AM];
        if constexpr (MHD) {
            b1p = ct[T_BP];
            b1m = ct[T_BM];
            b2p = rt[T_BP];
            b2m = rt[T_BM];
        }
    }
    static_assert(!(GEN && MHD), "the D2Q5 scheme runs on straight grids only");
    // 16-bit storage: reference entries of the own row (one row per wave:
    // lane 0 always holds a node of it, and lanes without a node store
    // nothing), read through scalar loads
    CPtr<float> rin = nullptr;
    if constexpr (Store<S>::scaled) rin = (CPtr<float>)(pl.ref_in + (d.row_off + jw) * kRef);
    T f[kQ], Fp1, Fp2;
    tile_pull9<S, T, FT>(d, b, planeF, ic, jc, rin, f, Fp1, Fp2);
    T dg[2][kM];   // D2Q5 deviations (MHD)
    const T sginv = Store<S>::scaled ? sp[P_ISCG] : T(1);
    if (mhd_run) pull_g<S, T>(d, b, ic, jc, sginv, rin, dg);
    if (ly * TX + (lx & ~63) < nh) {   // (uniform over the wave: whether its first lane has a ring node)
        T hf[kQ], hF1, hF2;
        const float* hrf = Store<S>::scaled ? pl.ref_in + (d.row_off + hj) * kRef : nullptr;
        tile_pull9<S, T, FT>(d, b, planeF, hi, hj, hrf, hf, hF1, hF2);
        const T hih1 = GEN ? ld_at<T>(mt + M_IH1 * NB, hnb) : ctab[hi * kTab + T_IH];
        const T hih2 = GEN ? ld_at<T>(mt + M_IH2 * NB, hnb) : rtab[hj * kTab + T_IH];
        T hdr, hU1, hU2;
        tile_moments<T>(hf, hF1, hF2, p.rho0, hih1, hih2, hdr, hU1, hU2);
        if (hv) {
            sm[0][hy + 1][hx + 1] = hdr;
            sm[1][hy + 1][hx + 1] = hU1;
            sm[2][hy + 1][hx + 1] = hU2;
        }
    }
    T dr, U1, U2;
    tile_moments<T>(f, Fp1, Fp2, p.rho0, g.ih1, g.ih2, dr, U1, U2);
    if (in) {
        sm[0][ly + 1][lx + 1] = dr;
        sm[1][ly + 1][lx + 1] = U1;
        sm[2][ly + 1][lx + 1] = U2;
    }
    __syncthreads();
    if (!in || i < ox || j < oy) return;

    const T rho = p.rho0 + dr;
    const int cx = lx + 1, cy = ly + 1;
    const T d1U1 = tile_fd<T>([&](int c) { return sm[1][cy][c]; }, cx, i, nx, px);
    const T d1r = tile_fd<T>([&](int c) { return sm[0][cy][c]; }, cx, i, nx, px);
    const T d2U2 = tile_fd<T>([&](int r) { return sm[2][r][cx]; }, cy, j, ny, py);
    const T d2r = tile_fd<T>([&](int r) { return sm[0][r][cx]; }, cy, j, ny, py);

    // (from here on every lane of the wave holds a node of row jw = j)
    const bool wxlo = !px && i == 0, wxhi = !px && i == nx - 1;
    // (forced to scalar registers: the compiler otherwise keeps these
    // row-uniform flags and the rows below in vector lanes)
    const bool wylo = __builtin_amdgcn_readfirstlane(int(!py && jw == 0)) != 0;
    const bool wyhi = __builtin_amdgcn_readfirstlane(int(!py && jw == ny - 1)) != 0;
    // 16-bit storage: the reference entries of rows j, j - 1 and j + 1 of the
    // output table (wrapped when periodic; a row beyond a wall is never a
    // reader's, so it is clamped into the grid)
    CPtr<float> R0 = nullptr, Rm = nullptr, Rp = nullptr;
    if constexpr (Store<S>::scaled) {
        const int jm = __builtin_amdgcn_readfirstlane(jw > 0 ? jw - 1 : (py ? ny - 1 : 0));
        const int jp = __builtin_amdgcn_readfirstlane(jw < ny - 1 ? jw + 1 : (py ? 0 : ny - 1));
        const CPtr<float> rt0 = (CPtr<float>)(pl.ref_out + d.row_off * kRef);
        R0 = rt0 + jw * kRef;
        Rm = rt0 + jm * kRef;
        Rp = rt0 + jp * kRef;
    }
    const uint32_t seed = mix32(step_ctr[0] + uint32_t(k));
    const uint32_t hn = mix32((uint32_t(d.f_off) + uint32_t(j) * uint32_t(d.pitch) + uint32_t(i)) ^ seed);
    const uint32_t cs = uint32_t(sizeof(S));
    const uint32_t own = uint32_t(j + 1) * b.pitch_s + uint32_t(i) * cs;   // (slot regions start at row -1)
    const bool bot = jw == 0, top = jw == ny - 1;
    // App. G, as the march: magnetic field, local derivatives, Lorentz
    // force, the D2Q5 collision and writes (stored value = base + increment;
    // anti-bounce-back slots negate the post-collision value; the writer adds
    // the rest-state offsets of the interior axis slots of component 2)
    T Fx1 = p.Fx1, Fx2 = p.Fx2;
    if (mhd_run) {
        T B1, B2, FL1, FL2, dgi[2][kM];
        mie_node<T>(p, g, dg, U1, U2, B1, B2, FL1, FL2, dgi);
        Fx1 += FL1;
        Fx2 += FL2;
        const T hh = g.h1 * g.h2;
#pragma unroll
        for (int a = 1; a < kM; ++a) {
            const int ex = ex_(a), ey = ey_(a);
            const bool wx = (ex > 0 && wxhi) || (ex < 0 && wxlo);
            const bool wy = (ey > 0 && wyhi) || (ey < 0 && wylo);
            if (wx || wy) {
                // the reader (this node) sees -g~ + 2 W h_wall B_wall with B_wall = (0, B0)
                const T hwall = wy ? g.h1 * sp[ey < 0 ? P_HWLO : P_HWHI] : sp[ex < 0 ? P_H1WLO : P_H1WHI] * g.h2;
                dg[0][a] = -dg[0][a];
                dgi[0][a] = -dgi[0][a];
                dg[1][a] = -dg[1][a];
                dgi[1][a] = -dgi[1][a] + T(2) * p.W1 * p.B0 * (hwall - hh);
            } else {
                dgi[1][a] += a == 1 ? g.h2 * b1p : a == 3 ? g.h2 * b1m : a == 2 ? g.h1 * b2p : g.h1 * b2m;
            }
        }
        const T sgw = Store<S>::scaled ? sp[P_SCG] : T(1);
        float rg[2][kM] = {};   // (16-bit) reference of each slot's reader
        if constexpr (Store<S>::scaled) {
#pragma unroll
            for (int ci = 0; ci < 2; ++ci)
                reader_refs<kM>(R0 + kRefG + ci * kM, Rm + kRefG + ci * kM, Rp + kRefG + ci * kM, wylo, wyhi,
                                rg[ci]);
            if (!px)   // (uniform: walls on the xi1 faces)
#pragma unroll
                for (int ci = 0; ci < 2; ++ci) xwall_refs<kM>(R0 + kRefG + ci * kM, rg[ci], wxlo, wxhi, dgi[ci]);
        }
        S eg[2][kM];
#pragma unroll
        for (int ci = 0; ci < 2; ++ci)
#pragma unroll
            for (int a = 0; a < kM; ++a) {
                eg[ci][a] = Store<S>::enc(Store<S>::scaled ? dg[ci][a] - rg[ci][a] : dg[ci][a], dgi[ci][a], sgw,
                                          pop_draw(hn, kQ + ci * kM + a));
                st_nt<NT, S>(b.go, ci * b.g_comp + uint32_t(a) * b.plane_s + own, eg[ci][a]);
            }
        // ghost rows: plane 2 / 4 of each component, own column
        if (bot || top) {
            const bool wall = !py;
            const uint32_t grow = (wall ? bot : top) ? 0u : uint32_t(ny + 1) * b.pitch_s;
            const uint32_t pg = (wall == bot) ? 2u : 4u;
#pragma unroll
            for (int ci = 0; ci < 2; ++ci)
                st_nt<NT, S>(b.go, grow + ci * b.g_comp + pg * b.plane_s + uint32_t(i) * cs, bot ? eg[ci][4] : eg[ci][2]);
        }
    }

    const RawDev<T> m = raw_dev<T>(f);
    T F1, F2, n3, n4, inc[kQ];
    if constexpr (GEN)
        force_and_corrections_gen<T>(p, g, rho, dr, U1, U2, d1U1, d2U2, d1r, d2r, p.Fx1, p.Fx2, m.m11, F1, F2,
                                     n3, n4);
    else
        force_and_corrections<T>(p, g, rho, dr, U1, U2, d1U1, d2U2, d1r, d2r, Fx1, Fx2, F1, F2, n3, n4);
    if constexpr (COLL == kCollRaw)
        raw_collide<T>(p, g, m, rho, dr, U1, U2, Fp1, Fp2, F1, F2, n3, n4, inc);
    else
        cm_collide<T>(p, g, m, rho, dr, U1, U2, Fp1, Fp2, F1, F2, n3, n4, inc);

    // writer side: rest-state offsets of the axis slots (their readers are the
    // neighbours; zero toward walls) and the wall terms of App. C
    if constexpr (GEN) {
        inc[1] += aE;
        inc[3] += aW;
        inc[2] += aN;
        inc[4] += aS;
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
    } else {   // the march's arithmetic: wall coefficients precomputed per run
        inc[1] += g.h2 * aE;
        inc[3] += g.h2 * aW;
        inc[2] += g.h1 * aN;
        inc[4] += g.h1 * aS;
        if (wyhi && d.uw_hi != 0.0) {
            const T cw = rho * sp[P_CWHI];
            if (d.lid_corners || !wxhi) inc[5] -= cw;
            if (d.lid_corners || !wxlo) inc[6] += cw;
        }
        if (wylo && d.uw_lo != 0.0) {
            const T cw = rho * sp[P_CWLO];
            if (d.lid_corners || !wxlo) inc[7] += cw;
            if (d.lid_corners || !wxhi) inc[8] -= cw;
        }
        if (wxhi && d.vw_hi != 0.0) {
            const T cx = rho * sp[P_CXHI];
            if (d.lid_corners || !wyhi) inc[5] -= cx;
            if (d.lid_corners || !wylo) inc[8] += cx;
        }
        if (wxlo && d.vw_lo != 0.0) {
            const T cx = rho * sp[P_CXLO];
            if (d.lid_corners || !wylo) inc[7] += cx;
            if (d.lid_corners || !wyhi) inc[6] -= cx;
        }
    }

    // stores: base + increment, rounded without bias (the same draws as the
    // straight march: node, population, step)
    // (16-bit storage: the reader's reference comes off the base first, then
    // the increment is added, so the rounded residual loses nothing to the
    // size of the reference)
    float ro[kQ] = {};
    if constexpr (Store<S>::scaled) {
        reader_refs<kQ>(R0, Rm, Rp, wylo, wyhi, ro);
        if (!px) xwall_refs<kQ>(R0, ro, wxlo, wxhi, inc);   // (uniform: walls on the xi1 faces)
    }
    S e[kQ];
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        const T sfw = Store<S>::scaled ? sp[P_SC + cls_(a)] : T(1);
        e[a] = Store<S>::enc(Store<S>::scaled ? f[a] - ro[a] : f[a], inc[a], sfw, pop_draw(hn, a));
        st_nt<NT, S>(b.fo, uint32_t(a) * b.plane_s + own, e[a]);
    }
    // ghost rows (rows 0 and ny - 1): walls take the bounced values at the
    // reader's source column, into the row beyond the wall; periodic xi2 takes
    // copies of the slots the opposite edge row pulls, into the ghost row
    // beyond that edge.  Planes: walls bottom {2, 5, 6}, top {4, 8, 7};
    // periodic bottom {4, 7, 8}, top {2, 6, 5}.
    if (bot || top) {
        const bool wall = !py;
        const uint32_t grow = (wall ? bot : top) ? 0u : uint32_t(ny + 1) * b.pitch_s;   // row -1 or ny
        const uint32_t p0 = (wall == bot) ? 2 : 4;
        const uint32_t p1 = wall ? (bot ? 5 : 8) : (bot ? 7 : 6);
        const uint32_t p2 = wall ? (bot ? 6 : 7) : (bot ? 8 : 5);
        const int cm = px ? (i == 0 ? nx - 1 : i - 1) : i - 1;
        const int cp = px ? (i == nx - 1 ? 0 : i + 1) : i + 1;
        st_nt<NT, S>(b.fo, grow + p0 * b.plane_s + uint32_t(i) * cs, bot ? e[4] : e[2]);
        if (!wall) {
            st_nt<NT, S>(b.fo, grow + p1 * b.plane_s + uint32_t(i) * cs, bot ? e[7] : e[6]);
            st_nt<NT, S>(b.fo, grow + p2 * b.plane_s + uint32_t(i) * cs, bot ? e[8] : e[5]);
        } else {
            if (!wxlo) st_nt<NT, S>(b.fo, grow + p1 * b.plane_s + uint32_t(cm) * cs, bot ? e[7] : e[6]);
            if (!wxhi) st_nt<NT, S>(b.fo, grow + p2 * b.plane_s + uint32_t(cp) * cs, bot ? e[8] : e[5]);
        }
    }
    const uint32_t nf = uint32_t(j) * b.pitch_F + uint32_t(i) * uint32_t(sizeof(FT));
    st_nt<NT, FT>(b.Fo, nf, FT(F1));
    st_nt<NT, FT>(b.Fo, nf + planeF, FT(F2));
}

}  // namespace goc
