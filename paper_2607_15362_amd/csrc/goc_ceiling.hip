// goc_ceiling.hip -- bandwidth instruments for the roofline of the tiled step
// (libgocceiling.so, declared in include/goc_ceiling.h).
//
// A measurement aid, not part of the method: the pattern kernel moves the
// bytes of one tiled time step (App. E: pull of every slot from its
// neighbour, writes of the node's own slots, of the ghost rows and of the
// lagged force; with the D2Q5 slots of App. G) in the library's layout and
// launch geometry, and computes nothing but a sum per pulled node.  Its
// duration bounds what the step can reach with this memory pattern; the copy
// kernel gives the plain one-stream figure beside it, and the mix kernel
// plain streams in other read / write proportions (HBM delivers less when
// reads and writes interleave).  All allocate their own buffers; nothing
// here is used by the step.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "goc_tile.hpp"
#include "../../include/goc_ceiling.h"
#include "../../include/goc_lbm.h"

namespace {

using goc::kTileX;

// The tiled step's memory traffic for one straight run: the same tile
// shape (TX x TY) and placement (XCD bands, partial edge tiles), the same pulls of the own
// node and of the ring around the tile (slot offsets of pull_off), one LDS
// value per pulled node and a barrier, and the same stores (nine slots, ten
// D2Q5 slots, the ghost rows of rows 0 and ny - 1, the two force planes).
// Raw storage values are moved unchanged: the stored slot is the own pulled
// slot plus the LDS sum of the left and right neighbours scaled by zero at
// run time (so that no load can be dropped).
template <class S, bool MHD, int TY, bool NT, int TX>
__global__ void __launch_bounds__(TX * TY)
pattern_kernel(goc::RunDesc d, goc::Pools<S, float> pl, float zero)
{
    using goc::kQ;
    using goc::kM;
    __shared__ float sm[TY + 2][TX + 2];
    const int nx = d.nx, ny = d.ny;
    const int gx = (nx + TX - 1) / TX, gy = (ny + TY - 1) / TY;
    const int nt = gx * gy;
    const int xcd = blockIdx.x & 7, q = nt >> 3, rem = nt & 7;
    const int t = xcd * q + min(xcd, rem) + (int)(blockIdx.x >> 3);
    const int ox = (t % gx) * TX, oy = (t / gx) * TY;
    const bool px = d.bc_x == 0, py = d.bc_y == 0;
    int tx, ty, x0, y0;
    goc::tile_span(nx, TX, ox, px, tx, x0);
    goc::tile_span(ny, TY, oy, py, ty, y0);
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int i = x0 + lx, j = y0 + ly;
    const bool in = lx < tx && ly < ty;
    const goc::RunBytes b = goc::run_bytes(d, pl);
    const uint32_t planeF = uint32_t(d.plane * sizeof(float));
    const int ic = in ? i : x0, jc = in ? j : y0;
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
    S f[kQ], g[2][kM];
    float F1, F2;
#pragma unroll
    for (int a = 0; a < kQ; ++a) f[a] = goc::ld_at<S>(b.f, goc::pull_off<S>(d, b, ic, jc, a));
    {
        const uint32_t nf = uint32_t(jc) * b.pitch_F + uint32_t(ic) * 4u;
        F1 = goc::ld_at<float>(b.F, nf);
        F2 = goc::ld_at<float>(b.F, nf + planeF);
    }
    if constexpr (MHD) {
#pragma unroll
        for (int a = 0; a < kM; ++a) {
            const uint32_t off = goc::pull_off<S>(d, b, ic, jc, a);
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) g[ci][a] = goc::ld_at<S>(b.g, ci * b.g_comp + off);
        }
    }
    if (ly * TX + (lx & ~63) < nh) {
        float s = 0.f;
#pragma unroll
        for (int a = 0; a < kQ; ++a) s += float(goc::ld_at<S>(b.f, goc::pull_off<S>(d, b, hi, hj, a)));
        const uint32_t nf = uint32_t(hj) * b.pitch_F + uint32_t(hi) * 4u;
        s += goc::ld_at<float>(b.F, nf) + goc::ld_at<float>(b.F, nf + planeF);
        if (hv) sm[hy + 1][hx + 1] = s;
    }
    if (in) {
        float s = F1 + F2;
#pragma unroll
        for (int a = 0; a < kQ; ++a) s += float(f[a]);
        sm[ly + 1][lx + 1] = s;
    }
    __syncthreads();
    if (!in || i < ox || j < oy) return;
    const float v = zero * (sm[ly + 1][lx] + sm[ly + 1][lx + 2]);
    const uint32_t cs = uint32_t(sizeof(S));
    const uint32_t own = uint32_t(j + 1) * b.pitch_s + uint32_t(i) * cs;
    const int jw = __builtin_amdgcn_readfirstlane(jc);
    const bool bot = jw == 0, top = jw == ny - 1;
    const S dv = S(v);
    if constexpr (MHD) {
#pragma unroll
        for (int ci = 0; ci < 2; ++ci)
#pragma unroll
            for (int a = 0; a < kM; ++a)
                goc::st_nt<NT, S>(b.go, ci * b.g_comp + uint32_t(a) * b.plane_s + own, S(g[ci][a] + dv));
        if (bot || top) {
            const bool wall = !py;
            const uint32_t grow = (wall ? bot : top) ? 0u : uint32_t(ny + 1) * b.pitch_s;
            const uint32_t pg = (wall == bot) ? 2u : 4u;
#pragma unroll
            for (int ci = 0; ci < 2; ++ci)
                goc::st_nt<NT, S>(b.go, grow + ci * b.g_comp + pg * b.plane_s + uint32_t(i) * cs,
                                  bot ? g[ci][4] : g[ci][2]);
        }
    }
#pragma unroll
    for (int a = 0; a < kQ; ++a) goc::st_nt<NT, S>(b.fo, uint32_t(a) * b.plane_s + own, S(f[a] + dv));
    if (bot || top) {
        const bool wall = !py;
        const bool wxlo = !px && i == 0, wxhi = !px && i == nx - 1;
        const uint32_t grow = (wall ? bot : top) ? 0u : uint32_t(ny + 1) * b.pitch_s;
        const uint32_t p0 = (wall == bot) ? 2 : 4;
        const uint32_t p1 = wall ? (bot ? 5 : 8) : (bot ? 7 : 6);
        const uint32_t p2 = wall ? (bot ? 6 : 7) : (bot ? 8 : 5);
        const int cm = px ? (i == 0 ? nx - 1 : i - 1) : i - 1;
        const int cp = px ? (i == nx - 1 ? 0 : i + 1) : i + 1;
        goc::st_nt<NT, S>(b.fo, grow + p0 * b.plane_s + uint32_t(i) * cs, bot ? f[4] : f[2]);
        if (!wall) {
            goc::st_nt<NT, S>(b.fo, grow + p1 * b.plane_s + uint32_t(i) * cs, bot ? f[7] : f[6]);
            goc::st_nt<NT, S>(b.fo, grow + p2 * b.plane_s + uint32_t(i) * cs, bot ? f[8] : f[5]);
        } else {
            if (!wxlo) goc::st_nt<NT, S>(b.fo, grow + p1 * b.plane_s + uint32_t(cm) * cs, bot ? f[7] : f[6]);
            if (!wxhi) goc::st_nt<NT, S>(b.fo, grow + p2 * b.plane_s + uint32_t(cp) * cs, bot ? f[8] : f[5]);
        }
    }
    const uint32_t nf = uint32_t(j) * b.pitch_F + uint32_t(i) * 4u;
    goc::st_nt<NT, float>(b.Fo, nf, F1 + v);
    goc::st_nt<NT, float>(b.Fo, nf + planeF, F2 + v);
}

// One-stream copy: 16-byte vectors, grid-stride, four loads in flight per
// thread before their stores.
__global__ void __launch_bounds__(256) copy_kernel(const float4* __restrict__ a, float4* __restrict__ o, int64_t n)
{
    const int64_t s = (int64_t)gridDim.x * 256;
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; k + 3 * s < n; k += 4 * s) {
        const float4 v0 = a[k], v1 = a[k + s], v2 = a[k + 2 * s], v3 = a[k + 3 * s];
        o[k] = v0;
        o[k + s] = v1;
        o[k + 2 * s] = v2;
        o[k + 3 * s] = v3;
    }
    for (; k < n; k += s) o[k] = a[k];
}

// Streams of 16-byte vectors in a chosen read / write mix: R input and W
// output buffers of n vectors each, element k of every output written from
// element k of every input, four elements in flight per thread, in one of
// two orders: grid-stride (the whole grid sweeps the buffers together) or
// CHUNK (each work-group sweeps a contiguous share of them on its own); with
// no output each thread folds what it reads into one value, written only if
// it matches a value the inputs never hold (so no load is dropped).
typedef float f4v __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ inline void st4(f4v* p, f4v v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int R, int W, bool NT, bool CHUNK>
__global__ void __launch_bounds__(256) mix_kernel(const f4v* __restrict__ a0, const f4v* __restrict__ a1,
                                                  f4v* __restrict__ o0, f4v* __restrict__ o1, int64_t n,
                                                  float* __restrict__ sink)
{
    // the elements [lo, hi) this thread's work-group covers, with stride s
    int64_t s = (int64_t)gridDim.x * 256, k = (int64_t)blockIdx.x * 256 + threadIdx.x, hi = n;
    if constexpr (CHUNK) {
        const int64_t per = (n + gridDim.x - 1) / gridDim.x, lo = (int64_t)blockIdx.x * per;
        hi = lo + per < n ? lo + per : n;
        s = 256;
        k = lo + threadIdx.x;
    }
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    auto in = [&](int64_t e) {
        f4v v = {1.f, 1.f, 1.f, 1.f};
        if constexpr (R >= 1) v = a0[e];
        if constexpr (R >= 2) v += a1[e];
        return v;
    };
    auto out = [&](int64_t e, f4v v) {
        if constexpr (W >= 1) st4<NT>(o0 + e, v);
        if constexpr (W >= 2) st4<NT>(o1 + e, v + 1.f);
        if constexpr (W == 0) acc += v;
    };
    for (; k + 3 * s < hi; k += 4 * s) {
        const f4v v0 = in(k), v1 = in(k + s), v2 = in(k + 2 * s), v3 = in(k + 3 * s);
        out(k, v0);
        out(k + s, v1);
        out(k + 2 * s, v2);
        out(k + 3 * s, v3);
    }
    for (; k < hi; k += s) out(k, in(k));
    if constexpr (W == 0)
        if (acc.x + acc.y + acc.z + acc.w == -1.f) sink[0] = acc.x;   // (the buffers hold zeros)
}

template <int R, int W, bool NT, bool CHUNK>
hipError_t launch_mix(int blocks, hipStream_t st, void* const* p, int64_t n, float* sink)
{
    hipLaunchKernelGGL((mix_kernel<R, W, NT, CHUNK>), dim3(blocks), dim3(256), 0, st,
                       static_cast<const f4v*>(p[0]), static_cast<const f4v*>(p[1]), static_cast<f4v*>(p[2]),
                       static_cast<f4v*>(p[3]), n, sink);
    return hipGetLastError();
}

template <int R, int W>
hipError_t launch_mix_nt(bool nt, bool chunk, int blocks, hipStream_t st, void* const* p, int64_t n, float* sink)
{
    if (chunk)
        return nt ? launch_mix<R, W, true, true>(blocks, st, p, n, sink)
                  : launch_mix<R, W, false, true>(blocks, st, p, n, sink);
    return nt ? launch_mix<R, W, true, false>(blocks, st, p, n, sink)
              : launch_mix<R, W, false, false>(blocks, st, p, n, sink);
}

struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events()
    {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

// Device buffers of one measurement, freed once the stream has drained (an
// error return may leave work in flight).
struct Buffers {
    hipStream_t st = nullptr;
    void* p[6] = {};
    explicit Buffers(hipStream_t s) : st(s) {}
    ~Buffers()
    {
        (void)hipStreamSynchronize(st);
        for (void* q : p)
            if (q) (void)hipFree(q);
    }
};

template <class S, bool MHD, int TY, bool NT, int TX>
int run_pattern(const goc::RunDesc& d, int64_t f_elems, int64_t F_elems, int reps, hipStream_t st, double* us)
{
    Buffers buf(st);
    const size_t fb = size_t(f_elems) * sizeof(S), Fb = size_t(F_elems) * sizeof(float);
    const size_t sizes[4] = {fb, fb, Fb, Fb};
    for (int k = 0; k < 4; ++k) {
        if (hipMalloc(&buf.p[k], sizes[k]) != hipSuccess) return GOC_ENOMEM;
        if (hipMemsetAsync(buf.p[k], 0, sizes[k], st) != hipSuccess) return GOC_EDEVICE;
    }
    const int gx = (d.nx + TX - 1) / TX, gy = (d.ny + TY - 1) / TY;
    const dim3 grid(gx * gy), block(TX, TY);
    auto launch = [&](int k) {
        goc::Pools<S, float> pl{};
        const int a = k & 1;
        pl.fin = static_cast<const S*>(buf.p[a]);
        pl.fout = static_cast<S*>(buf.p[1 - a]);
        pl.Fin = static_cast<const float*>(buf.p[2 + a]);
        pl.Fout = static_cast<float*>(buf.p[3 - a]);
        pl.gin = pl.fin;   // (the D2Q5 planes lie in the rows of the slot pool)
        pl.gout = pl.fout;
        hipLaunchKernelGGL((pattern_kernel<S, MHD, TY, NT, TX>), grid, block, 0, st, d, pl, 0.f);
        return hipGetLastError();
    };
    for (int k = 0; k < 4; ++k)
        if (launch(k) != hipSuccess) return GOC_EDEVICE;
    Events ev;
    if (hipEventCreate(&ev.e0) != hipSuccess || hipEventCreate(&ev.e1) != hipSuccess) return GOC_EDEVICE;
    if (hipEventRecord(ev.e0, st) != hipSuccess) return GOC_EDEVICE;
    for (int k = 0; k < reps; ++k)
        if (launch(k) != hipSuccess) return GOC_EDEVICE;
    if (hipEventRecord(ev.e1, st) != hipSuccess || hipEventSynchronize(ev.e1) != hipSuccess) return GOC_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess) return GOC_EDEVICE;
    *us = 1e3 * double(ms) / reps;
    return GOC_OK;
}

template <class S, bool MHD, int TY, int TX>
int pick_nt(const goc::RunDesc& d, int64_t fe, int64_t Fe, int nt, int reps, hipStream_t st, double* us)
{
    return nt ? run_pattern<S, MHD, TY, true, TX>(d, fe, Fe, reps, st, us)
              : run_pattern<S, MHD, TY, false, TX>(d, fe, Fe, reps, st, us);
}

template <class S, bool MHD>
int pick_shape(const goc::RunDesc& d, int64_t fe, int64_t Fe, int cols, int rows, int nt, int reps, hipStream_t st,
               double* us)
{
    if (cols == goc::kTileXWide) return pick_nt<S, MHD, goc::kTileRowsWide, goc::kTileXWide>(d, fe, Fe, nt, reps, st, us);
    switch (rows) {
    case 4: return pick_nt<S, MHD, 4, kTileX>(d, fe, Fe, nt, reps, st, us);
    case 8: return pick_nt<S, MHD, 8, kTileX>(d, fe, Fe, nt, reps, st, us);
    default: return pick_nt<S, MHD, 16, kTileX>(d, fe, Fe, nt, reps, st, us);
    }
}

}  // namespace

extern "C" int goc_ceiling_pattern(int nx, int ny, int mhd, int storage_bytes, int tile_cols, int tile_rows,
                                   int nontemporal, int reps, void* stream, double* us_per_launch)
{
    const bool narrow = tile_cols == kTileX && (tile_rows == 4 || tile_rows == 8 || tile_rows == 16);
    const bool wide = tile_cols == goc::kTileXWide && tile_rows == goc::kTileRowsWide;
    if (!us_per_launch || nx < 3 || ny < 3 || reps < 1 || (storage_bytes != 4 && storage_bytes != 2) ||
        !(narrow || wide))
        return GOC_EINVAL;
    goc::RunDesc d{};
    d.nx = nx;
    d.ny = ny;
    d.bc_x = GOC_BC_PERIODIC;
    d.bc_y = GOC_BC_WALL;
    d.mhd = mhd ? 1 : 0;
    const int64_t row = goc::padded_row(nx);
    d.plane = row;
    d.pitch = int32_t((mhd ? 2 * goc::kGPlanes : 9) * row);
    d.pitchF = int32_t(2 * row);
    const int64_t region = (int64_t)d.pitch * (ny + 2) + 256, regionF = (int64_t)d.pitchF * ny + 256;
    if (region * storage_bytes > (int64_t)UINT32_MAX) return GOC_EINVAL;
    d.f_off = d.pitch;
    d.g_off = d.pitch + (mhd ? goc::kGPlanes * row : 0);
    d.F_off = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nt = nontemporal ? 1 : 0;
    if (storage_bytes == 4)
        return mhd ? pick_shape<float, true>(d, region, regionF, tile_cols, tile_rows, nt, reps, st, us_per_launch)
                   : pick_shape<float, false>(d, region, regionF, tile_cols, tile_rows, nt, reps, st, us_per_launch);
    return mhd ? pick_shape<__half, true>(d, region, regionF, tile_cols, tile_rows, nt, reps, st, us_per_launch)
               : pick_shape<__half, false>(d, region, regionF, tile_cols, tile_rows, nt, reps, st, us_per_launch);
}

extern "C" int goc_ceiling_copy(int64_t bytes, int reps, void* stream, double* us_per_launch)
{
    if (!us_per_launch || bytes < 16 || bytes % 16 != 0 || reps < 1) return GOC_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Buffers buf(st);
    for (int k = 0; k < 2; ++k) {
        if (hipMalloc(&buf.p[k], size_t(bytes)) != hipSuccess) return GOC_ENOMEM;
        if (hipMemsetAsync(buf.p[k], 0, size_t(bytes), st) != hipSuccess) return GOC_EDEVICE;
    }
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    const int64_t n = bytes / 16;
    const int blocks = 32 * ncu;
    auto launch = [&](int k) {
        hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, st, static_cast<const float4*>(buf.p[k & 1]),
                           static_cast<float4*>(buf.p[1 - (k & 1)]), n);
        return hipGetLastError();
    };
    for (int k = 0; k < 4; ++k)
        if (launch(k) != hipSuccess) return GOC_EDEVICE;
    Events ev;
    if (hipEventCreate(&ev.e0) != hipSuccess || hipEventCreate(&ev.e1) != hipSuccess) return GOC_EDEVICE;
    if (hipEventRecord(ev.e0, st) != hipSuccess) return GOC_EDEVICE;
    for (int k = 0; k < reps; ++k)
        if (launch(k) != hipSuccess) return GOC_EDEVICE;
    if (hipEventRecord(ev.e1, st) != hipSuccess || hipEventSynchronize(ev.e1) != hipSuccess) return GOC_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess) return GOC_EDEVICE;
    *us_per_launch = 1e3 * double(ms) / reps;
    return GOC_OK;
}

extern "C" int goc_ceiling_mix(int64_t bytes, int reads, int writes, int nontemporal, int chunked, int wg_per_cu,
                               int reps, void* stream, double* us_per_launch)
{
    if (!us_per_launch || bytes < 16 || bytes % 16 != 0 || reads < 0 || reads > 2 || writes < 0 || writes > 2 ||
        reads + writes < 1 || (nontemporal != 0 && nontemporal != 1) || (chunked != 0 && chunked != 1) ||
        wg_per_cu < 1 || wg_per_cu > 64 || reps < 1)
        return GOC_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Buffers buf(st);
    // p[0], p[1]: inputs; p[2], p[3]: outputs; p[4]: the sink
    const int used[4] = {reads >= 1, reads >= 2, writes >= 1, writes >= 2};
    for (int k = 0; k < 4; ++k) {
        if (!used[k]) continue;
        if (hipMalloc(&buf.p[k], size_t(bytes)) != hipSuccess) return GOC_ENOMEM;
        if (hipMemsetAsync(buf.p[k], 0, size_t(bytes), st) != hipSuccess) return GOC_EDEVICE;
    }
    if (hipMalloc(&buf.p[4], 16) != hipSuccess) return GOC_ENOMEM;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) ncu = prop.multiProcessorCount;
    }
    const int64_t n = bytes / 16;
    const int blocks = wg_per_cu * ncu;
    float* sink = static_cast<float*>(buf.p[4]);
    const bool nt = nontemporal != 0, ch = chunked != 0;
    auto launch = [&]() -> hipError_t {
        switch (reads * 3 + writes) {
            case 1: return launch_mix_nt<0, 1>(nt, ch, blocks, st, buf.p, n, sink);
            case 2: return launch_mix_nt<0, 2>(nt, ch, blocks, st, buf.p, n, sink);
            case 3: return launch_mix_nt<1, 0>(nt, ch, blocks, st, buf.p, n, sink);
            case 4: return launch_mix_nt<1, 1>(nt, ch, blocks, st, buf.p, n, sink);
            case 5: return launch_mix_nt<1, 2>(nt, ch, blocks, st, buf.p, n, sink);
            case 6: return launch_mix_nt<2, 0>(nt, ch, blocks, st, buf.p, n, sink);
            case 7: return launch_mix_nt<2, 1>(nt, ch, blocks, st, buf.p, n, sink);
            default: return launch_mix_nt<2, 2>(nt, ch, blocks, st, buf.p, n, sink);
        }
    };
    for (int k = 0; k < 4; ++k)
        if (launch() != hipSuccess) return GOC_EDEVICE;
    Events ev;
    if (hipEventCreate(&ev.e0) != hipSuccess || hipEventCreate(&ev.e1) != hipSuccess) return GOC_EDEVICE;
    if (hipEventRecord(ev.e0, st) != hipSuccess) return GOC_EDEVICE;
    for (int k = 0; k < reps; ++k)
        if (launch() != hipSuccess) return GOC_EDEVICE;
    if (hipEventRecord(ev.e1, st) != hipSuccess || hipEventSynchronize(ev.e1) != hipSuccess) return GOC_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.e0, ev.e1) != hipSuccess) return GOC_EDEVICE;
    *us_per_launch = 1e3 * double(ms) / reps;
    return GOC_OK;
}
