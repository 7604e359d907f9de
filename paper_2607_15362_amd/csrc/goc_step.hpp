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

// (written with selects, no branches: the step kernel calls these for every
// row on scalar values)
__device__ inline bool row_ok(const RunDesc& d, int r) { return (d.bc_y == 0) | (uint32_t(r) < uint32_t(d.ny)); }
// Rows within two of the domain (all the step asks for), wrapped when periodic.
__device__ inline int row_wrap(const RunDesc& d, int r)
{
    const int w = r < 0 ? r + d.ny : (r >= d.ny ? r - d.ny : r);
    return d.bc_y != 0 ? r : w;
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
        const int64_t n = d.F_off + (int64_t)r * d.pitchF + L.col;
        Fp1 = T(Fin[n]);
        Fp2 = T(Fin[n + d.plane]);
    }
    dr = m00 * ih1 * ih2;
    const T irho = recip_sum(rho0, dr);
    U1 = (m10 + T(0.5) * Fp1) * ih2 * irho;
    U2 = (m01 + T(0.5) * Fp2) * ih1 * irho;
}

// Rounding draws of a node's populations (D2Q9 populations 0-8, then the
// ten D2Q5 populations): the low 24 bits of the node hash hn times distinct
// odd 24-bit multipliers (a full-rate 24-bit multiply), whose high result
// bits are the dither.
__device__ inline uint32_t pop_draw(uint32_t hn, int a)
{
    return __umul24(hn, (0x9E3779u * uint32_t(2 * a + 1)) & 0xFFFFFFu | 1u);
}

// Metric table of the compute type: the FP64 tables for FP64 arithmetic,
// their FP32 copy otherwise.
// Read-only memory read at wave-uniform addresses (constant address space).
template <class T> using CPtr = const __attribute__((address_space(4))) T*;

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

// Buffer resource over `bytes` bytes from `base` (raw 32-bit format).  The
// hardware range-checks every lane's byte offset against `bytes`: beyond it
// a load returns zero and a store writes nothing.  The step kernel issues
// all its loads and stores unconditionally and turns the unneeded ones off
// this way (bytes = 0 for a row it does not need, an offset of kOff for a
// lane that owns no node): with no branch around any memory instruction,
// the waits for a row's loads never include the loads issued after them.
// bytes < 2^32: the library refuses larger runs at creation, so kOff lies
// beyond every resource.
constexpr uint32_t kOff = 0xFFFFFFFFu;
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, __builtin_bit_cast(int, bytes),
                                             0x00020000);
}
template <class S>
__device__ inline S buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    const int o = __builtin_bit_cast(int, off);
    if constexpr (sizeof(S) == 2) {
        return __builtin_bit_cast(S, (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, o, 0, 0));
    } else if constexpr (sizeof(S) == 4) {
        return __builtin_bit_cast(S, (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0));
    } else {
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
    }
}
template <class S>
__device__ inline void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t off, S v)
{
    const int o = __builtin_bit_cast(int, off);
    if constexpr (sizeof(S) == 2) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, o, 0, 0);
    } else if constexpr (sizeof(S) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, o, 0, 0);
    } else {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, o, 0, 0);
    }
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

// Byte addressing of one run's pool regions (a region is below 4 GiB, so
// every offset within it fits in 32 bits).  The slot regions (f, g) start at
// ghost row -1: row r begins (r + 1) rows in, and rows -1 and ny hold the
// slots the pulls of rows 0 and ny - 1 take from beyond the domain in y
// (the writers of those rows fill them).
struct RunBytes {
    const char *f, *F, *g;           // input regions (slots from row -1, lagged force, D2Q5 from row -1)
    char *fo, *Fo, *go;              // output regions
    uint32_t pitch_s, pitch_F;       // one row of the slot / force regions
    uint32_t plane_s;                // one plane within a row
    uint32_t f_all, F_all, g_all;    // region sizes (ny + 2, ny and ny + 2 rows)
    uint32_t g_comp;                 // one D2Q5 component: 5 planes of a row
    int ny;
};

template <class S, class FT>
__device__ inline RunBytes run_bytes(const RunDesc& d, const Pools<S, FT>& pl)
{
    RunBytes b;
    b.f = reinterpret_cast<const char*>(pl.fin + (d.f_off - d.pitch));
    b.F = reinterpret_cast<const char*>(pl.Fin + d.F_off);
    b.g = reinterpret_cast<const char*>(pl.gin + (d.g_off - d.pitch));
    b.fo = reinterpret_cast<char*>(pl.fout + (d.f_off - d.pitch));
    b.Fo = reinterpret_cast<char*>(pl.Fout + d.F_off);
    b.go = reinterpret_cast<char*>(pl.gout + (d.g_off - d.pitch));
    b.pitch_s = uint32_t(d.pitch * sizeof(S));
    b.pitch_F = uint32_t(d.pitchF * sizeof(FT));
    b.plane_s = uint32_t(d.plane * sizeof(S));
    b.f_all = uint32_t((int64_t)d.pitch * (d.ny + 2) * sizeof(S));
    b.F_all = uint32_t((int64_t)d.pitchF * d.ny * sizeof(FT));
    // (the D2Q5 planes start g_off - f_off elements into the rows of the slot
    // pool: their region ends where the pool's does)
    b.g_all = b.f_all - uint32_t((d.g_off - d.f_off) * (int64_t)sizeof(S));
    b.g_comp = uint32_t(kM * d.plane * sizeof(S));
    b.ny = d.ny;
    return b;
}

// Issue the loads of the nine slots pulled into row r and of its lagged
// force (byte offsets offF[2] of the lane's node in the two force planes);
// valid = false issues them with an empty resource (zeros, no memory
// access).  Every direction's source row is uniform (rows -1 and ny are the
// ghost rows), so a slot is the lane's constant byte offset off[a] (plane,
// source row relative to row r - 1, column; see the kernel) from the base
// of row r - 1: one code path for every row.
template <class S, class FT>
__device__ inline void issue_row(const RunBytes& b, const uint32_t* off, const uint32_t* offF, int r, bool valid,
                                 S* raw, FT* Fr)
{
    const int rv = valid ? r : 0;
    const uint32_t e0 = uint32_t(rv) * b.pitch_s;   // row r - 1 (regions start at row -1)
    const __amdgpu_buffer_rsrc_t rs = rsrc(b.f + e0, valid ? b.f_all - e0 : 0u);
#pragma unroll
    for (int a = 0; a < kQ; ++a) raw[a] = buf_ld<S>(rs, off[a]);
    const uint32_t eF = uint32_t(rv) * b.pitch_F;
    const __amdgpu_buffer_rsrc_t rF = rsrc(b.F + eF, valid ? b.F_all - eF : 0u);
    Fr[0] = buf_ld<FT>(rF, offF[0]);
    Fr[1] = buf_ld<FT>(rF, offF[1]);
}

// The same for the ten D2Q5 slots of row r (component planes ci kM + a).
template <class S>
__device__ inline void issue_row_g(const RunBytes& b, const uint32_t* off, int r, bool valid, S (*graw)[kM])
{
    const int rv = valid ? r : 0;
    const uint32_t e0 = uint32_t(rv) * b.pitch_s;
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) {
        const uint32_t e = ci * b.g_comp + e0;
        const __amdgpu_buffer_rsrc_t rs = rsrc(b.g + e, valid ? b.g_all - e : 0u);
#pragma unroll
        for (int a = 0; a < kM; ++a) graw[ci][a] = buf_ld<S>(rs, off[a]);
    }
}

// Issue the loads of the halo node of lanes 0 and 63 in row r (the node
// beside the strip that the differences along xi1 need): its nine pulled
// slots and the first component of its lagged force.  hoff / hoffF are the
// offsets from the kernel, kOff (off) for every other lane and where no halo
// node is needed; valid = false issues none.
template <class S, class FT>
__device__ inline void issue_halo(const RunBytes& b, const uint32_t* hoff, uint32_t hoffF, int r, bool valid,
                                  S* hraw, FT& hF)
{
    const int rv = valid ? r : 0;
    const uint32_t e0 = uint32_t(rv) * b.pitch_s;
    const __amdgpu_buffer_rsrc_t rs = rsrc(b.f + e0, valid ? b.f_all - e0 : 0u);
#pragma unroll
    for (int a = 0; a < kQ; ++a) hraw[a] = buf_ld<S>(rs, hoff[a]);
    const uint32_t eF = uint32_t(rv) * b.pitch_F;
    hF = buf_ld<FT>(rsrc(b.F + eF, valid ? b.F_all - eF : 0u), hoffF);
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
// A wave owns 64 columns (one per lane, starting at a multiple of 64) and a
// segment of rows, and marches up the rows with four row slots (rows j-1,
// j, j+1, j+2); the loads of rows j+2 and j+3 are in flight while row j is
// collided.  Lanes 0 and 63 also pull the node beside the strip, one row
// ahead, for the differences along xi1.  COLL selects the collision body
// (kCollCentral or kCollRaw) for every run of the launch.
template <class S, bool MHD, int COLL>
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
    const bool own = craw >= x0 && craw < x1;
    const bool xwall_lo = d.bc_x != 0 && L.col == 0;
    const bool xwall_hi = d.bc_x != 0 && L.col == d.nx - 1;
    const T* ctab = table_of<T>(pl.col, pl.colf) + (int64_t)(d.col_off + Ls.col) * kTab;
    // the row tables are read at wave-uniform indices through the constant
    // address space: scalar loads, which the wave waits for on their own
    // counter instead of behind the population loads in flight
    const CPtr<T> rtab = (CPtr<T>)(table_of<T>(pl.row, pl.rowf) + (int64_t)d.row_off * kTab);
    const T h1_0 = ctab[T_H], ih1_0 = ctab[T_IH], th11_0 = ctab[T_TH];
    const T a1p_0 = ctab[T_AP], a1m_0 = ctab[T_AM], b1p_0 = ctab[T_BP], b1m_0 = ctab[T_BM];
    // per-lane pull offsets of interior rows in bytes, relative to the base
    // of row r - 1: plane a, the source row r - ey and the source column, or
    // through an x-wall the lane's own node (row r) in the opposite plane.
    // All are non-negative and below 2^32.
    uint32_t off[kQ];
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        const int ex = ex_(a), ey = ey_(a);
        int64_t e;
        if (ex == 0) {
            e = (int64_t)a * d.plane + (1 - ey) * d.pitch + Ls.col;
        } else {
            const bool wx = ex > 0 ? Ls.wm : Ls.wp;
            e = wx ? (int64_t)opp_(a) * d.plane + d.pitch + Ls.col
                   : (int64_t)a * d.plane + (1 - ey) * d.pitch + (ex > 0 ? Ls.cm : Ls.cp);
        }
        off[a] = uint32_t(e * (int64_t)sizeof(S));
    }
    const uint32_t offF[2] = {uint32_t(Ls.col * sizeof(FT)),     // the two force planes
                              uint32_t((d.plane + Ls.col) * sizeof(FT))};
    // halo nodes of the differences along xi1: the column left of lane 0 and
    // right of lane 63 (wrapped when periodic; none beyond a wall, where the
    // one-sided difference is used), pulled like an own node by that lane
    const bool hl = lane == 0, hr = lane == kWave - 1;
    const LaneCol Lh = lane_col(d, hl ? craw - 1 : craw + 1);
    const bool hneed = (hl || hr) && Lh.valid;
    uint32_t hoff[kQ];
#pragma unroll
    for (int a = 0; a < kQ; ++a) {
        const int ex = ex_(a), ey = ey_(a);
        int64_t e;
        if (ex == 0) {
            e = (int64_t)a * d.plane + (1 - ey) * d.pitch + Lh.col;
        } else {
            const bool wx = ex > 0 ? Lh.wm : Lh.wp;
            e = wx ? (int64_t)opp_(a) * d.plane + d.pitch + Lh.col
                   : (int64_t)a * d.plane + (1 - ey) * d.pitch + (ex > 0 ? Lh.cm : Lh.cp);
        }
        hoff[a] = hneed ? uint32_t(e * (int64_t)sizeof(S)) : kOff;
    }
    const uint32_t hoffF = hneed ? uint32_t(Lh.col * sizeof(FT)) : kOff;
    const T ih1h = table_of<T>(pl.col, pl.colf)[(int64_t)(d.col_off + (hneed ? Lh.col : Ls.col)) * kTab + T_IH];
    const RunBytes rb = run_bytes(d, pl);
    // byte offsets of the writes from the base of output row j: plane and own
    // column; kOff (discarded) for lanes that own no node
    uint32_t wf[kQ], wF[2], wg[MHD ? 2 * kM : 1];
#pragma unroll
    for (int a = 0; a < kQ; ++a) wf[a] = own ? uint32_t(((int64_t)a * d.plane + L.col) * sizeof(S)) : kOff;
#pragma unroll
    for (int c = 0; c < 2; ++c) wF[c] = own ? uint32_t(((int64_t)c * d.plane + L.col) * sizeof(FT)) : kOff;
    if constexpr (MHD) {
#pragma unroll
        for (int a = 0; a < 2 * kM; ++a) wg[a] = own ? uint32_t(((int64_t)a * d.plane + L.col) * sizeof(S)) : kOff;
    }
    // ghost-row writes of rows 0 and ny - 1: offsets within a plane row.
    // Walls: the source column of the reader's pull (own column, or for the
    // diagonal slots the neighbour's; none where the reader bounces in x
    // instead); periodic: the own column (copies).
    const uint32_t gw0 = own ? uint32_t(L.col * sizeof(S)) : kOff;
    const uint32_t gw1 = !own ? kOff : d.bc_y != 0 ? (L.wm ? kOff : uint32_t(L.cm * sizeof(S))) : gw0;
    const uint32_t gw2 = !own ? kOff : d.bc_y != 0 ? (L.wp ? kOff : uint32_t(L.cp * sizeof(S))) : gw0;
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
    // one resource per plane of output row j: the row's bytes (0: none)
    // resource over a pool from output row j to its end (nplanes planes); no
    // bytes when off
    // (slot regions start at ghost row -1: row j is j + 1 rows in)
    auto out_row = [&](char* region, uint32_t pitch, uint32_t all, int row_in, bool on) {
        const uint32_t e = uint32_t(row_in) * pitch;
        return rsrc(region + e, on ? all - e : 0u);
    };

    int y0, y1;
    seg_rows(d.ny, d.segs, seg, y0, y1);

    // window: A = row y0 - 1, B = row y0, C = row y0 + 1 and D = row y0 + 2
    // (loads in flight)
    // (a row outside a walled domain is loaded as zeros and never used)
    Slot A, B, C, D;
    const bool ok_a = row_ok(d, y0 - 1);
    const int ra = ok_a ? row_wrap(d, y0 - 1) : y0;
    issue_row<S, FT>(rb, off, offF, ra, ok_a, A.raw, A.Fr);
    issue_row<S, FT>(rb, off, offF, y0, true, B.raw, B.Fr);
    issue_row<S, FT>(rb, off, offF, row_wrap(d, y0 + 1), row_ok(d, y0 + 1), C.raw, C.Fr);
    issue_row<S, FT>(rb, off, offF, row_wrap(d, y0 + 2), y0 + 2 <= y1 && row_ok(d, y0 + 2),
                     D.raw, D.Fr);
    // D2Q5 slots of the segment's rows only (each row reads its own)
    if constexpr (MHD) {
        issue_row_g<S>(rb, off, y0, mhd_run, B.graw);
        issue_row_g<S>(rb, off, row_wrap(d, y0 + 1), mhd_run && y0 + 1 < y1, C.graw);
        issue_row_g<S>(rb, off, row_wrap(d, y0 + 2), mhd_run && y0 + 2 < y1, D.graw);
    }
    S hraw[kQ];   // halo node of the next row (lanes 0 and 63)
    FT hF;
    issue_halo<S, FT>(rb, hoff, hoffF, y0, true, hraw, hF);
    // All four rows are in flight together; draining them here, once per
    // segment, leaves nothing of the set-up pending at the loop entry, so the
    // compiler's waits inside the loop follow the steady state (each row's
    // loads waited for two rows after their issue) instead of the set-up's
    // more recent loads.
    __builtin_amdgcn_s_waitcnt(0);
    decode_row<S, T, FT>(A, sinv, p0.rho0, ih1_0, ih2_of(ra));
    decode_row<S, T, FT>(B, sinv, p0.rho0, ih1_0, ih2_of(y0));

    const int64_t plane = d.plane;
    // one row: P = row j - 1, Cs = row j, N = row j + 1, Q = row j + 2 (its
    // loads in flight; its moments still those of row j - 2)
    auto row_step = [&](Slot& P, Slot& Cs, Slot& N, Slot& Q, int j) {
        // the scheduler keeps each row to itself (interleaving the unrolled
        // rows only lengthens live ranges); the loads issued here complete
        // during the row's arithmetic
        __builtin_amdgcn_sched_barrier(0);
        // The run's scalars (parameters, byte sizes, scales) are read again
        // for every row, through a pointer the compiler cannot follow from
        // one row to the next: they come from the scalar cache instead of
        // occupying scalar registers through the whole march, which made the
        // compiler spill them into vector lanes.
        CPtr<RunDesc> drow = (CPtr<RunDesc>)&d;
        asm volatile("" : "+s"(drow));
        const RunDesc& d = *(const RunDesc*)drow;
        const NodeParams<T> p = node_params<T>(d);
        const RunBytes rb = run_bytes(d, pl);
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
        // per-row opaque copies of the lane constants
        T h1 = h1_0, ih1 = ih1_0, th11 = th11_0, a1p = a1p_0, a1m = a1m_0, b1p = b1p_0, b1m = b1m_0;
        opaque_v(h1);
        opaque_v(ih1);
        opaque_v(th11);
        opaque_v(a1p);
        opaque_v(a1m);
        opaque_v(b1p);
        opaque_v(b1m);
        const bool act = j < y1;             // a row of this segment (else stores off)
        const int jt = min(j, d.ny - 1);     // table row (rows beyond the domain read the last)
        // 0. the halo node of row j (its loads were issued one row earlier,
        //    before those of row j + 2), decoded as decode_row does; then
        //    the halo loads of row j + 1
        T hU, hR;
        {
            const T ih2j = rtab[(int64_t)jt * kTab + T_IH];
            T hf[kQ];
#pragma unroll
            for (int a = 0; a < kQ; ++a) hf[a] = Store<S>::dec(hraw[a], sinv[cls_(a)]);
            const T m00 = ((hf[0] + hf[1]) + (hf[2] + hf[3])) + ((hf[4] + hf[5]) + (hf[6] + hf[7])) + hf[8];
            const T m10 = (hf[1] - hf[3]) + ((hf[5] - hf[6]) + (hf[8] - hf[7]));
            hR = m00 * ih1h * ih2j;
            const T irho = recip_sum(p.rho0, hR);
            hU = (m10 + T(0.5) * T(hF)) * ih2j * irho;
        }
        // (kept here: decoded later, the halo registers would have to be
        // duplicated while the next row's halo is in flight)
        opaque_v(hU);
        opaque_v(hR);
        __builtin_amdgcn_sched_barrier(0);
        issue_halo<S, FT>(rb, hoff, hoffF, row_wrap(d, j + 1), j + 1 < y1 && row_ok(d, j + 1), hraw,
                          hF);
        // (the halo loads go out first: the wait for them one row later then
        // leaves the loads of row j + 3 in flight)
        __builtin_amdgcn_sched_barrier(0);
        // 1. loads of row j + 3 (into P, whose populations are done)
        const bool have_next = row_ok(d, j + 1);
        issue_row<S, FT>(rb, off, offF, row_wrap(d, j + 3), j + 3 <= y1 && row_ok(d, j + 3),
                         P.raw, P.Fr);
        if constexpr (MHD)
            issue_row_g<S>(rb, off, row_wrap(d, j + 3), mhd_run && j + 3 < y1, P.graw);
        // 2. moments of row j + 1
        decode_row<S, T, FT>(N, sinv, p.rho0, ih1, ih2_of(have_next ? min(row_wrap(d, j + 1), d.ny - 1) : jt));

        NodeMetric<T> g;
        g.h1 = h1;
        g.ih1 = ih1;
        g.th11 = th11;
        const CPtr<T> rt = rtab + (int64_t)jt * kTab;
        g.h2 = rt[T_H];
        g.ih2 = rt[T_IH];
        g.th22 = rt[T_TH];
        // 3. differences along xi2 (one-sided next to walls)
        T d2U2, d2r;
        // (the rows these need are in the march: no load here, as a load in
        // a branch would make the compiler's later waits conservative)
        if (d.bc_y != 0 && j == 0) {
            // row 2: the raw slots of Q (the segment starts at row 0, so
            // they were loaded, and waited for, at its set-up)
            Slot W;
#pragma unroll
            for (int a = 0; a < kQ; ++a) W.raw[a] = Q.raw[a];
            W.Fr[0] = Q.Fr[0];
            W.Fr[1] = Q.Fr[1];
            decode_row<S, T, FT>(W, sinv, p.rho0, ih1, ih2_of(2));
            d2U2 = T(0.5) * (T(-3) * Cs.U2 + T(4) * N.U2 - W.U2);
            d2r = T(0.5) * (T(-3) * Cs.dr + T(4) * N.dr - W.dr);
        } else if (d.bc_y != 0 && j == d.ny - 1) {
            // row ny - 3: the moments Q still holds (the top segment has at
            // least four rows, or starts at row 0 when ny = 3)
            d2U2 = T(0.5) * (T(3) * Cs.U2 - T(4) * P.U2 + Q.U2);
            d2r = T(0.5) * (T(3) * Cs.dr - T(4) * P.dr + Q.dr);
        } else {
            d2U2 = T(0.5) * (N.U2 - P.U2);
            d2r = T(0.5) * (N.dr - P.dr);
        }
        // differences along xi1 from the neighbouring lanes
        const T drho = Cs.dr, rho = p.rho0 + drho, U1 = Cs.U1, U2 = Cs.U2;
        // (the lane shifts run with every lane active: a shift inside a
        // lane-divergent branch would read inactive lanes)
        // (the shifts are pinned before the halo values replace them in lanes
        // 0 and 63: folded into the selects, the compiler would shift under a
        // mask without lanes 0 / 63, and their neighbours would then read the
        // halo value instead of the lane's own)
        T Um1 = from_prev(U1), Up1 = from_next(U1), rm1 = from_prev(drho), rp1 = from_next(drho);
        opaque_v(Um1);
        opaque_v(Up1);
        opaque_v(rm1);
        opaque_v(rp1);
        Um1 = hl ? hU : Um1;
        Up1 = hr ? hU : Up1;
        rm1 = hl ? hR : rm1;
        rp1 = hr ? hR : rp1;
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
        //    anti-bounce-back slots negate the post-collision value)
        T Fx1 = p.Fx1, Fx2 = p.Fx2;
        const RowGeo Gj = row_geo(d, j);
        const int64_t nn = (int64_t)j * d.pitch + L.col;
        const uint32_t hn = mix32(uint32_t(d.f_off + nn) ^ seed);
        if constexpr (MHD) {   // (a plain run of a mixed batch: no D2Q5 memory access, no force)
            T dg[2][kM], dgi[2][kM];
#pragma unroll
            for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                for (int a = 0; a < kM; ++a) dg[ci][a] = T(Store<S>::dec(Cs.graw[ci][a], sginv));
            T B1, B2, FL1, FL2;
            mie_node<T>(p, g, dg, U1, U2, B1, B2, FL1, FL2, dgi);
            if (mhd_run) {
                Fx1 += FL1;
                Fx2 += FL2;
            }
            {
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
                const __amdgpu_buffer_rsrc_t rg = out_row(rb.go, rb.pitch_s, rb.g_all, j + 1, mhd_run && act);
                S eg[2][kM];
#pragma unroll
                for (int ci = 0; ci < 2; ++ci)
#pragma unroll
                    for (int a = 0; a < kM; ++a) {
                        eg[ci][a] = Store<S>::enc(dg[ci][a], dgi[ci][a], sgw, pop_draw(hn, kQ + ci * kM + a));
                        buf_st<S>(rg, wg[ci * kM + a], eg[ci][a]);
                    }
                // ghost rows (as for the populations below): plane 2 / 4 of
                // each component, own column
                const bool bot = j == 0, top = j == d.ny - 1, wall = d.bc_y != 0;
                const bool on = mhd_run && act && (bot || top);
                const uint32_t eg_row = (wall ? bot : top) ? 0u : uint32_t(d.ny + 1) * rb.pitch_s;
                const uint32_t pg = (wall == bot) ? 2u : 4u;
#pragma unroll
                for (int ci = 0; ci < 2; ++ci)
                    buf_st<S>(rsrc(rb.go + eg_row + (ci * kM + pg) * rb.plane_s, on ? rb.plane_s : 0u), gw0,
                              bot ? eg[ci][4] : eg[ci][2]);
            }
        }

        // 5. effective force, corrections, central-moment collision
        T F1, F2, n3, n4, inc[kQ];
        force_and_corrections<T>(p, g, rho, drho, U1, U2, d1U1, d2U2, d1r, d2r, Fx1, Fx2, F1, F2, n3, n4);
        if constexpr (COLL == kCollRaw)
            raw_collide<T>(p, g, raw_dev<T>(Cs.f), rho, drho, U1, U2, Cs.Fp1, Cs.Fp2, F1, F2, n3, n4, inc);
        else
            cm_collide<T>(p, g, raw_dev<T>(Cs.f), rho, drho, U1, U2, Cs.Fp1, Cs.Fp2, F1, F2, n3, n4, inc);

        // 6. D2Q9 writes: inc holds the collision increments; the writer adds the
        //    rest-state offsets of the interior axis slots (the reader is the
        //    neighbour; its rest state differs through the metric) and the
        //    reader's wall terms
        {
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
            // the same for walls on the xi1 faces moving along xi2 (at a
            // corner, with lid_corners, the terms of both walls add)
            if (xwall_hi && d.vw_hi != 0.0) {
                const T cx = rho * sp[P_CXHI];
                // slot 5 is read back as f7, slot 8 as f6: f7 = ft5 - cx, f6 = ft8 + cx
                if (d.lid_corners || !Gj.wp) inc[5] -= cx;
                if (d.lid_corners || !Gj.wm) inc[8] += cx;
            }
            if (xwall_lo && d.vw_lo != 0.0) {
                const T cx = rho * sp[P_CXLO];
                // slot 7 is read back as f5, slot 6 as f8: f5 = ft7 + cx, f8 = ft6 - cx
                if (d.lid_corners || !Gj.wm) inc[7] += cx;
                if (d.lid_corners || !Gj.wp) inc[6] -= cx;
            }
            const __amdgpu_buffer_rsrc_t rf = out_row(rb.fo, rb.pitch_s, rb.f_all, j + 1, act);
            S e[kQ];
#pragma unroll
            for (int a = 0; a < kQ; ++a) {
                e[a] = Store<S>::enc(Cs.f[a], inc[a], sfw[cls_(a)], pop_draw(hn, a));
                buf_st<S>(rf, wf[a], e[a]);
            }
            // ghost rows: the writers of rows 0 and ny - 1 also store, into
            // row -1 or ny, the three slots their own row's pulls take from
            // beyond the domain in y.  Walls: the bounced value (the slot of
            // the opposite direction, which already holds the reader's wall
            // terms) at the reader's source column, into the row beyond the
            // wall; periodic: copies of the slots the opposite edge row pulls,
            // into the ghost row beyond that edge.  Planes: walls bottom
            // {2, 5, 6}, top {4, 8, 7}; periodic bottom {4, 7, 8}, top {2, 6, 5}.
            {
                const bool bot = j == 0, top = j == d.ny - 1, wall = d.bc_y != 0;
                const bool on = act && (bot || top);
                const uint32_t eg_row = (wall ? bot : top) ? 0u : uint32_t(d.ny + 1) * rb.pitch_s;
                const uint32_t p0 = (wall == bot) ? 2u : 4u;
                const uint32_t p1 = wall ? (bot ? 5u : 8u) : (bot ? 7u : 6u);
                const uint32_t p2 = wall ? (bot ? 6u : 7u) : (bot ? 8u : 5u);
                const uint32_t nb = on ? rb.plane_s : 0u;
                buf_st<S>(rsrc(rb.fo + eg_row + p0 * rb.plane_s, nb), gw0, bot ? e[4] : e[2]);
                buf_st<S>(rsrc(rb.fo + eg_row + p1 * rb.plane_s, nb), gw1, bot ? e[7] : e[6]);
                buf_st<S>(rsrc(rb.fo + eg_row + p2 * rb.plane_s, nb), gw2, bot ? e[8] : e[5]);
            }
            const __amdgpu_buffer_rsrc_t rF = out_row(rb.Fo, rb.pitch_F, rb.F_all, j, act);
            buf_st<FT>(rF, wF[0], FT(F1));
            buf_st<FT>(rF, wF[1], FT(F2));
        }
        __builtin_amdgcn_sched_barrier(0);
    };

    // march with the four slots rotating roles (no moves between rows), a
    // group of four rows per pass.  The loop has a single exit and no code
    // after it that reads the slots: an exit from inside the body, or slots
    // live after the loop, would make the compiler join states at the loop
    // entry or copy the slots there, and every wait would then include the
    // loads in flight.  A segment is whole groups except at the top of the
    // domain; rows of a group beyond the segment run with their stores off.
    static_assert(kRowGroup == 4, "the march below unrolls four rows");
    for (int j = y0; j < y1; j += 4) {
        row_step(A, B, C, D, j);
        row_step(B, C, D, A, j + 1);
        row_step(C, D, A, B, j + 2);
        row_step(D, A, B, C, j + 3);
    }
}

}  // namespace goc
