// goc_aux.hpp -- once-per-run and read-out kernels: metric precompute,
// column / row tables, initial state, slot <-> population conversion,
// fields and global sums.  One thread per node (or per column / row); none
// of these is on the per-step path.
#pragma once

#include "goc_step.hpp"

namespace goc {

// Metric precompute in FP64: theta = (dh/dxi) / h^2 (Sec. 2.1, diagonal
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

// Column (or row) tables in FP64 (and an FP32 copy) from h and theta along
// one axis:
// h, 1/h, theta, P0/2 (1/h(i) - 1/h(i+-1)), W1 B0 (h(i) - h(i+-1)); the
// neighbour terms are zero where the neighbour lies beyond a wall (the slot
// is then read back by the node itself) and wrap when periodic.
__global__ void table_kernel(const double* __restrict__ h, const double* __restrict__ th, int n,
                             int periodic, double P0, double W1B0, double* __restrict__ tab,
                             float* __restrict__ tabf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ip = periodic ? (i + 1) % n : i + 1;
    const int im = periodic ? (i + n - 1) % n : i - 1;
    const bool hp = ip < n, hm = im >= 0;
    double* t = tab + (int64_t)i * kTab;
    t[T_H] = h[i];
    t[T_IH] = 1.0 / h[i];
    t[T_TH] = th[i];
    t[T_AP] = hp ? 0.5 * P0 * (1.0 / h[i] - 1.0 / h[ip]) : 0.0;
    t[T_AM] = hm ? 0.5 * P0 * (1.0 / h[i] - 1.0 / h[im]) : 0.0;
    t[T_BP] = hp ? W1B0 * (h[i] - h[ip]) : 0.0;
    t[T_BM] = hm ? W1B0 * (h[i] - h[im]) : 0.0;
    t[7] = 0.0;
    for (int k = 0; k < kTab; ++k) tabf[(int64_t)i * kTab + k] = float(t[k]);
}

// Destination slot of population a arriving at node (i, j): the slot its
// pull reads (inverse of the gather of the step kernel).
__device__ inline int64_t slot_index(const RunDesc& d, int i, int j, int a)
{
    int si = i - ex_(a), sj = j - ey_(a), pa = a;
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
    return (int64_t)pa * d.plane + (int64_t)sj * d.pitch + si;
}

// The ghost slot (row -1 or ny of the slot region) from which the step kernel
// pulls direction a into node (i, j), when that pull leaves the domain in y
// and does not bounce back through an x-wall first; false otherwise.  For
// a y-wall it holds what slot_index gives (the bounced value), for periodic y
// a copy of the wrapped slot.
__device__ inline bool ghost_index(const RunDesc& d, int i, int j, int a, int64_t& idx)
{
    const int sj = j - ey_(a);
    if (sj >= 0 && sj < d.ny) return false;
    int si = i - ex_(a);
    if (si < 0 || si >= d.nx) {
        if (d.bc_x != 0) return false;
        si = si < 0 ? si + d.nx : si - d.nx;
    }
    idx = (int64_t)a * d.plane + (int64_t)sj * d.pitch + si;
    return true;
}

// Store the deviation of population a of node (i, j) at the slot its pull
// reads (and at the step kernel's ghost copy of it).
template <class S, class T>
__device__ inline void put_slot(S* base, const RunDesc& d, int i, int j, int a, T v, T s)
{
    Store<S>::st(base, slot_index(d, i, j, a), v, s);
    int64_t gi;
    if (ghost_index(d, i, j, a, gi)) Store<S>::st(base, gi, v, s);
}

// Reference entry k of row j of run d in the table in use (16-bit storage;
// zero otherwise): what the stored value of a slot whose reader lies in
// row j leaves out.
template <class S, class FT>
__device__ inline double ref_of(const Pools<S, FT>& pl, const RunDesc& d, int j, int k)
{
    if constexpr (Store<S>::scaled) return double(pl.ref_in[(d.row_off + j) * kRef + k]);
    return 0.0;
}

__device__ inline double sc_of(const RunDesc& d, int a, bool scaled) { return scaled ? d.sc[cls_(a)] : 1.0; }

// Per-node metric of run d (FP64): the column / row tables of a straight
// grid, or the node planes of a general 2-D metric.
struct NodeM {
    double h1, h2, ih1, ih2, th11, th12, th21, th22;
};
template <class S, class FT>
__device__ inline NodeM node_metric(const RunDesc& d, const Pools<S, FT>& pl, int i, int j)
{
    NodeM m;
    if (d.metric2d) {
        const int64_t N = (int64_t)d.nx * d.ny;
        const double* q = pl.met + d.met_off + (int64_t)j * d.nx + i;
        m.h1 = q[M_H1 * N];
        m.ih1 = q[M_IH1 * N];
        m.h2 = q[M_H2 * N];
        m.ih2 = q[M_IH2 * N];
        m.th11 = q[M_TH11 * N];
        m.th12 = q[M_TH12 * N];
        m.th21 = q[M_TH21 * N];
        m.th22 = q[M_TH22 * N];
        return m;
    }
    const double* ct = pl.col + (d.col_off + i) * kTab;
    const double* rt = pl.row + (d.row_off + j) * kTab;
    m.h1 = ct[T_H];
    m.ih1 = ct[T_IH];
    m.th11 = ct[T_TH];
    m.h2 = rt[T_H];
    m.ih2 = rt[T_IH];
    m.th22 = rt[T_TH];
    m.th12 = m.th21 = 0.0;
    return m;
}

// Deviations from the rest state of the initial populations of node (i, j)
// (App. C): the raw equilibria of Sec. 3 with the corrections of Sec. 4
// (finite-difference gradients of the fields) mapped through P^-1; D2Q5 (dg
// not null): g^eq(0) of App. G.  Fields: FP64 [ny][nx] (rho_in nullptr: the
// rest state rho0, U = 0; b1_in nullptr: the applied field B = (0, B0)).
template <class S>
__device__ inline void init_devs(const RunDesc& d, const Pools<S, typename ForceOf<S>::type>& pl, int i, int j,
                                 const double* __restrict__ rho_in, const double* __restrict__ u1_in,
                                 const double* __restrict__ u2_in, const double* __restrict__ b1_in,
                                 const double* __restrict__ b2_in, typename ComputeOf<S>::type* f,
                                 typename ComputeOf<S>::type (*dgo)[kM])
{
    using T = typename ComputeOf<S>::type;
    const NodeParams<T> p = node_params<T>(d);
    const NodeM nm = node_metric(d, pl, i, j);
    NodeMetric<T> g;
    g.h1 = T(nm.h1);
    g.ih1 = T(nm.ih1);
    g.th11 = T(nm.th11);
    g.h2 = T(nm.h2);
    g.ih2 = T(nm.ih2);
    g.th22 = T(nm.th22);
    g.th12 = T(nm.th12);
    g.th21 = T(nm.th21);
    auto at = [&](const double* a, int ii, int jj) -> T { return T(a[(int64_t)jj * d.nx + ii]); };
    T rho = p.rho0, U1 = T(0), U2 = T(0), d1U1 = T(0), d2U2 = T(0), d1r = T(0), d2r = T(0);
    T drho = T(0);
    if (rho_in) {
        rho = at(rho_in, i, j);
        drho = T(rho_in[(int64_t)j * d.nx + i] - d.rho0);
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
    if (d.metric2d)   // (the corrections need tau^c only, not tau12)
        force_and_corrections_gen<T>(p, g, rho, drho, U1, U2, d1U1, d2U2, d1r, d2r, p.Fx1, p.Fx2, rho * U1 * U2,
                                     F1, F2, n3, n4);
    else
        force_and_corrections<T>(p, g, rho, drho, U1, U2, d1U1, d2U2, d1r, d2r, p.Fx1, p.Fx2, F1, F2, n3, n4);
    // raw-equilibrium deviations from the rest moments
    const T r21 = g.h2 * g.ih1, r12 = g.h1 * g.ih2, cs2 = p.cs2;
    const T dP = drho * cs2;
    const T k2s = r21 * (rho * U1 * U1 + dP) + r12 * (rho * U2 * U2 + dP) + n3;
    const T k2d = r21 * (rho * U1 * U1 + dP) - r12 * (rho * U2 * U2 + dP) + n4;
    const T m00 = g.h1 * g.h2 * drho, m10 = g.h2 * rho * U1, m01 = g.h1 * rho * U2;
    const T m20 = T(0.5) * (k2s + k2d), m02 = T(0.5) * (k2s - k2d);
    const T m11 = rho * U1 * U2;
    const T m21 = rho * (cs2 + U1 * U1) * U2 * g.ih1;
    const T m12 = rho * (cs2 + U2 * U2) * U1 * g.ih2;
    const T m22 = drho * cs2 * cs2 + rho * cs2 * (U1 * U1 + U2 * U2) + rho * U1 * U1 * U2 * U2;
    f[0] = m00 - m20 - m02 + m22;
    f[1] = T(0.5) * (m10 + m20 - m12 - m22);
    f[2] = T(0.5) * (m01 + m02 - m21 - m22);
    f[3] = T(0.5) * (-m10 + m20 + m12 - m22);
    f[4] = T(0.5) * (-m01 + m02 + m21 - m22);
    f[5] = T(0.25) * (m11 + m21 + m12 + m22);
    f[6] = T(0.25) * (-m11 + m21 - m12 + m22);
    f[7] = T(0.25) * (m11 - m21 - m12 + m22);
    f[8] = T(0.25) * (-m11 - m21 + m12 + m22);
    if (!dgo) return;
    T dB[2] = {T(0), T(0)};   // deviation of B from the applied field (0, B0)
    if (b1_in) {
        dB[0] = T(b1_in[(int64_t)j * d.nx + i]);
        dB[1] = T(b2_in[(int64_t)j * d.nx + i] - d.B0);
    }
    const T B[2] = {dB[0], p.B0 + dB[1]};
    const T U[2] = {U1, U2};
    for (int ci = 0; ci < 2; ++ci) {
        const T A1 = U[0] * B[ci] - B[0] * U[ci];
        const T A2 = U[1] * B[ci] - B[1] * U[ci];
        for (int a = 0; a < kM; ++a) {
            const T W = a == 0 ? p.W0 : p.W1;
            // g^eq(0) minus the rest state W h1 h2 B_rest
            dgo[ci][a] = W * (g.h1 * g.h2 * dB[ci] + (T(ex_(a)) * g.h2 * A1 + T(ey_(a)) * g.h1 * A2) * p.inv_csm2);
        }
    }
}

// Store the node deviations of row j of run d, given by dev(i, f, dg), at the
// slots their pulls read.  16-bit storage: the work-group first forms the row
// means of the deviations (FP64, fixed order), writes them as the row's
// entries of the reference table ref_tab (the table in use) and stores each
// deviation minus its mean.  One work-group of 256 threads per row.
template <class S, class Dev>
__device__ inline void store_row(const RunDesc& d, const Pools<S, typename ForceOf<S>::type>& pl, int j,
                                 float* __restrict__ ref_tab, Dev dev)
{
    using T = typename ComputeOf<S>::type;
    constexpr int nk = kRefG + 2 * kM;
    __shared__ float ref[kRef];
    if constexpr (Store<S>::scaled) {
        __shared__ double sh[nk][256];
        double acc[nk];
        for (int k = 0; k < nk; ++k) acc[k] = 0.0;
        for (int i = threadIdx.x; i < d.nx; i += blockDim.x) {
            T f[kQ], dg[2][kM] = {};
            dev(i, f, d.mhd ? dg : nullptr);
            for (int a = 0; a < kQ; ++a) acc[a] += double(f[a]);
            for (int ci = 0; ci < 2; ++ci)
                for (int a = 0; a < kM; ++a) acc[kRefG + ci * kM + a] += double(dg[ci][a]);
        }
        for (int k = 0; k < nk; ++k) sh[k][threadIdx.x] = acc[k];
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s)
                for (int k = 0; k < nk; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x < kRef) {
            const float v = threadIdx.x < nk ? float(sh[threadIdx.x][0] / d.nx) : 0.0f;
            ref[threadIdx.x] = v;
            ref_tab[(d.row_off + j) * kRef + threadIdx.x] = v;
        }
        __syncthreads();
    } else {
        if (threadIdx.x < kRef) ref[threadIdx.x] = 0.0f;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < d.nx; i += blockDim.x) {
        T f[kQ], dg[2][kM];
        dev(i, f, d.mhd ? dg : nullptr);
        for (int a = 0; a < kQ; ++a)
            put_slot<S, T>(pl.fout + d.f_off, d, i, j, a, f[a] - T(ref[a]), T(sc_of(d, a, Store<S>::scaled)));
        if (d.mhd) {
            const T sg = Store<S>::scaled ? T(d.scg) : T(1);
            for (int ci = 0; ci < 2; ++ci)
                for (int a = 0; a < kM; ++a)
                    put_slot<S, T>(pl.gout + d.g_off + ci * kM * d.plane, d, i, j, a,
                                   dg[ci][a] - T(ref[kRefG + ci * kM + a]), sg);
        }
    }
}

// Initial state of App. C from node fields (rho, U1, U2) and, for MHD runs,
// (B1, B2) (see init_devs), stored with the reference table of the 16-bit
// storage formed from it; lagged force zero.  Grid: one work-group of 256
// threads per row of run `run`.
template <class S>
__global__ void __launch_bounds__(256) init_kernel(const RunDesc* __restrict__ runs, int run,
                                                   Pools<S, typename ForceOf<S>::type> pl, float* __restrict__ ref_tab,
                                                   const double* __restrict__ rho_in, const double* __restrict__ u1_in,
                                                   const double* __restrict__ u2_in, const double* __restrict__ b1_in,
                                                   const double* __restrict__ b2_in)
{
    using T = typename ComputeOf<S>::type;
    using FT = typename ForceOf<S>::type;
    const RunDesc& d = runs[run];
    const int j = blockIdx.x;
    if (j >= d.ny) return;
    store_row<S>(d, pl, j, ref_tab, [&](int i, T* f, T (*dg)[kM]) {
        init_devs<S>(d, pl, i, j, rho_in, u1_in, u2_in, b1_in, b2_in, f, dg);
    });
    for (int i = threadIdx.x; i < d.nx; i += blockDim.x) {
        const int64_t n = (int64_t)j * d.pitchF + i;   // force pool
        pl.Fout[d.F_off + n] = FT(0);
        pl.Fout[d.F_off + n + d.plane] = FT(0);
    }
}

// Post-stream populations f = deviation + rest state of the node (the
// reader), FP64 node arrays f[9][ny][nx], F[2][ny][nx], g[10][ny][nx].
template <class S>
__global__ void gather_kernel(const RunDesc* __restrict__ runs, int run, Pools<S, typename ForceOf<S>::type> pl,
                              double* __restrict__ f, double* __restrict__ F, double* __restrict__ g)
{
    const RunDesc& d = runs[run];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const NodeM m = node_metric(d, pl, i, j);
    const int64_t N = (int64_t)d.nx * d.ny, o = (int64_t)j * d.nx + i;
    const bool sc = Store<S>::scaled;
    for (int a = 0; a < kQ; ++a) {
        const double dv = double(Store<S>::ld(pl.fin + d.f_off, slot_index(d, i, j, a), 1.0f)) / sc_of(d, a, sc) +
                          ref_of(pl, d, j, a);
        f[a * N + o] = dv + rest_pop(a, m.h1, m.h2, d.rho0, d.cs2);
    }
    const int64_t n = (int64_t)j * d.pitchF + i;   // force pool
    F[o] = double(pl.Fin[d.F_off + n]);
    F[N + o] = double(pl.Fin[d.F_off + n + d.plane]);
    if (d.mhd && g) {
        const double scg = sc ? d.scg : 1.0;
        for (int ci = 0; ci < 2; ++ci)
            for (int a = 0; a < kM; ++a) {
                const double dv = double(Store<S>::ld(pl.gin + d.g_off + ci * kM * d.plane,
                                                      slot_index(d, i, j, a), 1.0f)) / scg +
                                  ref_of(pl, d, j, kRefG + ci * kM + a);
                const double W = a == 0 ? 1.0 - 2.0 * d.csm2 : 0.5 * d.csm2;
                g[(ci * kM + a) * N + o] = dv + (ci == 1 ? W * m.h1 * m.h2 * d.B0 : 0.0);
            }
    }
}

// Populations given as FP64 node arrays (as gather_kernel writes them)
// stored as deviations from the rest state (with the reference table of the
// 16-bit storage formed from them).  One work-group of 256 threads per row.
template <class S>
__global__ void __launch_bounds__(256) scatter_kernel(const RunDesc* __restrict__ runs, int run,
                                                      Pools<S, typename ForceOf<S>::type> pl, float* __restrict__ ref_tab,
                                                      const double* __restrict__ f, const double* __restrict__ F,
                                                      const double* __restrict__ g)
{
    using T = typename ComputeOf<S>::type;
    using FT = typename ForceOf<S>::type;
    const RunDesc& d = runs[run];
    const int j = blockIdx.x;
    if (j >= d.ny) return;
    const int64_t N = (int64_t)d.nx * d.ny;
    store_row<S>(d, pl, j, ref_tab, [&](int i, T* fo, T (*dg)[kM]) {
        const NodeM m = node_metric(d, pl, i, j);
        const int64_t o = (int64_t)j * d.nx + i;
        for (int a = 0; a < kQ; ++a) fo[a] = T(f[a * N + o] - rest_pop(a, m.h1, m.h2, d.rho0, d.cs2));
        if (dg)
            for (int ci = 0; ci < 2; ++ci)
                for (int a = 0; a < kM; ++a) {
                    const double W = a == 0 ? 1.0 - 2.0 * d.csm2 : 0.5 * d.csm2;
                    dg[ci][a] = T(g[(ci * kM + a) * N + o] - (ci == 1 ? W * m.h1 * m.h2 * d.B0 : 0.0));
                }
    });
    for (int i = threadIdx.x; i < d.nx; i += blockDim.x) {
        const int64_t o = (int64_t)j * d.nx + i, n = (int64_t)j * d.pitchF + i;   // force pool
        pl.Fout[d.F_off + n] = FT(F[o]);
        pl.Fout[d.F_off + n + d.plane] = FT(F[N + o]);
    }
}

// Deviations of node (i, j) pulled from the input buffer.
template <class S, class T>
__device__ inline void node_devs(const RunDesc& d, const Pools<S, typename ForceOf<S>::type>& pl, int i, int j,
                                 T* f, T (*dg)[kM])
{
    const bool sc = Store<S>::scaled;
    for (int a = 0; a < kQ; ++a)
        f[a] = Store<S>::ld(pl.fin + d.f_off, slot_index(d, i, j, a), T(1.0 / sc_of(d, a, sc))) +
               T(ref_of(pl, d, j, a));
    if (dg)
        for (int ci = 0; ci < 2; ++ci)
            for (int a = 0; a < kM; ++a)
                dg[ci][a] = Store<S>::ld(pl.gin + d.g_off + ci * kM * d.plane, slot_index(d, i, j, a),
                                         T(sc ? 1.0 / d.scg : 1.0)) +
                            T(ref_of(pl, d, j, kRefG + ci * kM + a));
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
    const NodeM nm = node_metric(d, pl, i, j);
    T f[kQ], dg[2][kM];
    node_devs<S, T>(d, pl, i, j, f, d.mhd ? dg : nullptr);
    LaneCol L;
    L.col = i;
    L.valid = true;
    T dr, U1, U2, Fp1, Fp2;
    row_moments<typename ForceOf<S>::type, T>(d, pl.Fin, L, j, f, T(d.rho0), T(nm.ih1), T(nm.ih2), dr,
                                              U1, U2, Fp1, Fp2);
    const int64_t N = (int64_t)d.nx * d.ny, o = (int64_t)j * d.nx + i;
    if (rho_o) rho_o[o] = d.rho0 + double(dr);
    if (u_o) {
        u_o[o] = double(U1);
        u_o[N + o] = double(U2);
    }
    if (d.mhd && B_o) {
        double S1 = 0, S2 = 0;
        for (int a = 0; a < kM; ++a) {
            S1 += double(dg[0][a]);
            S2 += double(dg[1][a]);
        }
        const double ihh = nm.ih1 * nm.ih2;
        B_o[o] = S1 * ihh;
        B_o[N + o] = d.B0 + S2 * ihh;
    }
}

// Global sums (FP64 accumulation): each work-group of 256 threads strides
// over the nodes of run `run` (node idx, idx + 256 gridDim.x, ...) and
// writes one partial: [0] sum f, [1] sum h2 rho U1, [2] sum h1 rho U2,
// [3] sum h1 h2 B1, [4] sum h1 h2 B2, [5] max |U|, [6] non-finite count.
// The grid is at most kDiagBlocks work-groups, so the partials never exceed
// kDiagBlocks * kDiag doubles.
constexpr int kDiag = 7;
constexpr int kDiagBlocks = 4096;
template <class S>
__global__ void __launch_bounds__(256) diag_kernel(const RunDesc* __restrict__ runs, int run,
                                                   Pools<S, typename ForceOf<S>::type> pl, double* __restrict__ part)
{
    using T = typename ComputeOf<S>::type;
    __shared__ double sh[kDiag][256];
    const RunDesc& d = runs[run];
    const int64_t N = (int64_t)d.nx * d.ny;
    double v[kDiag] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < N;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx % d.nx), j = (int)(idx / d.nx);
        const NodeM nm = node_metric(d, pl, i, j);
        T f[kQ], dg[2][kM];
        node_devs<S, T>(d, pl, i, j, f, d.mhd ? dg : nullptr);
        LaneCol L;
        L.col = i;
        L.valid = true;
        T dr, U1, U2, Fp1, Fp2;
        row_moments<typename ForceOf<S>::type, T>(d, pl.Fin, L, j, f, T(d.rho0), T(nm.ih1), T(nm.ih2),
                                                  dr, U1, U2, Fp1, Fp2);
        const double rho = d.rho0 + double(dr);
        const double h1 = nm.h1, h2 = nm.h2;
        double m = h1 * h2 * d.rho0;   // sum of the rest-state populations
        int bad = 0;
        for (int a = 0; a < kQ; ++a) {
            m += double(f[a]);
            bad += isfinite(double(f[a])) ? 0 : 1;
        }
        v[0] += m;
        v[1] += h2 * rho * double(U1);
        v[2] += h1 * rho * double(U2);
        if (d.mhd) {
            double S1 = 0, S2 = 0;
            for (int a = 0; a < kM; ++a) {
                S1 += double(dg[0][a]);
                S2 += double(dg[1][a]);
                bad += (isfinite(double(dg[0][a])) ? 0 : 1) + (isfinite(double(dg[1][a])) ? 0 : 1);
            }
            v[3] += S1;
            v[4] += h1 * h2 * d.B0 + S2;
        }
        const double um = sqrt(double(U1) * double(U1) + double(U2) * double(U2));
        if (isfinite(um)) v[5] = fmax(v[5], um);
        else bad += 1;
        v[6] += bad;
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

// Second pass over the partials (one work-group), fixed order:
// deterministic.  Writes the eight outputs of goc_lbm_diagnostics: the sums
// of [0] - [2], the mean flow rate [3] = [1] / nx, the fluxes, max |U| and
// the non-finite count.
__global__ void diag_final_kernel(const double* __restrict__ part, int nparts, int nx, double* __restrict__ out)
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
    if (threadIdx.x == 0) {
        out[0] = sh[0][0];
        out[1] = sh[1][0];
        out[2] = sh[2][0];
        out[3] = sh[1][0] / nx;
        out[4] = sh[3][0];
        out[5] = sh[4][0];
        out[6] = sh[5][0];
        out[7] = sh[6][0];
    }
}

// New reference table of the 16-bit storage (written to ref_new) from the
// current state, decoded with the table in use: entry k of a row is the mean
// over the row of the deviation its nodes pull along direction k (FP64
// sums, rounded to FP32 once).  One work-group of 256 threads per row of
// every run (grid = the rows of all runs; a run's rows start at row_off).
template <class S>
__global__ void __launch_bounds__(256) ref_kernel(const RunDesc* __restrict__ runs, int nruns,
                                                  Pools<S, typename ForceOf<S>::type> pl, float* __restrict__ ref_new)
{
    using T = typename ComputeOf<S>::type;
    constexpr int nk = kRefG + 2 * kM;
    __shared__ double sh[nk][256];
    const int gr = blockIdx.x;
    int lo = 0, hi = nruns - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (runs[mid].row_off <= gr) lo = mid;
        else hi = mid - 1;
    }
    const RunDesc& d = runs[lo];
    const int j = gr - (int)d.row_off;
    double acc[nk];
    for (int k = 0; k < nk; ++k) acc[k] = 0.0;
    for (int i = threadIdx.x; i < d.nx; i += blockDim.x) {
        T f[kQ], dg[2][kM];
        node_devs<S, T>(d, pl, i, j, f, d.mhd ? dg : nullptr);
        for (int a = 0; a < kQ; ++a) acc[a] += double(f[a]);
        if (d.mhd)
            for (int ci = 0; ci < 2; ++ci)
                for (int a = 0; a < kM; ++a) acc[kRefG + ci * kM + a] += double(dg[ci][a]);
    }
    for (int k = 0; k < nk; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < nk; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < kRef)
        ref_new[(int64_t)gr * kRef + threadIdx.x] = threadIdx.x < nk ? float(sh[threadIdx.x][0] / d.nx) : 0.0f;
}

// dst[0 .. n) = src[0 .. n) (the new reference table taking over).
__global__ void copy_kernel(const float* __restrict__ src, float* __restrict__ dst, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k];
}

// Step counter of the rounding draws: set, or advanced after a block of
// steps (one thread; part of the captured step graphs).
__global__ void counter_kernel(uint32_t* __restrict__ c, uint32_t v, int add)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) c[0] = add ? c[0] + v : v;
}

}  // namespace goc
