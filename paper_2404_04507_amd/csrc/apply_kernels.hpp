// apply_kernels.hpp - the IWFPM Hamiltonian apply on gfx950 (device code).
//
//   H~ psi = Lambda psi + F* diag(V/N) F*^{-1} psi        (Sec. 4.1, eq:F)
//
// psi lives on the lifted grid K*_{K,L} (Sec. 3.2).  The index-shift
// transform T (Sec. 3.3) only relabels entries, so the transforms run on the
// rectangular grid and T appears in two places only: the gather of a
// window-ordered vector into grid order before the inverse FFT (T^{-1}), and
// the scatter after the forward FFT, where the true label k = rho^{-1}(k*)
// (eq:inverse1-3) is rebuilt on the fly for the diagonal kinetic term
// Lambda = 1/2 |2 pi P k|^2.
//
// Schedules
//   fused      one workgroup holds a whole vector in LDS: load + gather,
//              inverse transform along every axis, potential product,
//              forward transforms, kinetic term + scatter.  For small grids.
//   three-pass the grid axes are split into a trailing group (contiguous
//              slabs) and a leading group (strided columns):
//              pass 1  gather + inverse DFT along the trailing axes
//              pass 2  inverse DFT along the leading axes, x V, forward DFT
//              pass 3  forward DFT along the trailing axes + kinetic + scatter
//              with the intermediate kept in a plan-owned workspace.
// In every schedule the last inverse axis, the potential product and the
// first forward axis are fused in registers.
//
// Every 1-D transform is one pencil per thread (fft_reg.hpp); LDS holds the
// tile between axes.  The potential is either a sum of per-axis tables
// (all modes on coordinate axes, the common case) or a full grid.

#pragma once

#include <hip/hip_runtime.h>

#include "fft_reg.hpp"
#include "internal.hpp"
#include "sizes.hpp"

namespace iwfpm {

// ---------------------------------------------------------------------------
// pencils
// ---------------------------------------------------------------------------

template <int S, int SIGN, typename R>
__device__ __forceinline__ void pencil_fft(cplx<R>* base, int es) {
    cplx<R> x[S];
#pragma unroll
    for (int i = 0; i < S; ++i) x[i] = base[i * es];
    fft_inplace<S, SIGN>(x);
#pragma unroll
    for (int i = 0; i < S; ++i) base[i * es] = x[i];
}

template <typename R>
struct VPencil {
    const R* vgrid;     // potential grid (vmode 1) or nullptr
    const R* vaxis;     // table of the pencil's own axis (vmode 0)
    R vb;               // sum of the other axes' tables at this pencil (vmode 0)
    int gbase, gstep;   // grid index of element i: gbase + i * gstep (vmode 1)
};

// inverse DFT, times V, forward DFT, for one pencil
template <int S, typename R>
__device__ __forceinline__ void pencil_conv(cplx<R>* base, int es, const VPencil<R>& vp) {
    cplx<R> x[S];
#pragma unroll
    for (int i = 0; i < S; ++i) x[i] = base[i * es];
    fft_inplace<S, +1>(x);
    if (vp.vgrid) {
#pragma unroll
        for (int i = 0; i < S; ++i) x[i] = cscale(x[i], vp.vgrid[vp.gbase + i * vp.gstep]);
    } else {
#pragma unroll
        for (int i = 0; i < S; ++i) x[i] = cscale(x[i], vp.vb + vp.vaxis[i]);
    }
    fft_inplace<S, -1>(x);
#pragma unroll
    for (int i = 0; i < S; ++i) base[i * es] = x[i];
}

template <int SIGN, typename R, int MAXS>
__device__ __forceinline__ void dispatch_fft(int S, cplx<R>* base, int es) {
    switch (S) {
#define IWFPM_CASE(s) \
    case s:                                                       \
        if constexpr (s <= MAXS) pencil_fft<s, SIGN, R>(base, es); \
        break;
        IWFPM_EXTENTS(IWFPM_CASE)
#undef IWFPM_CASE
        default: break;  // the plan rejects extents outside IWFPM_EXTENTS
    }
}

template <typename R, int MAXS>
__device__ __forceinline__ void dispatch_conv(int S, cplx<R>* base, int es, const VPencil<R>& vp) {
    switch (S) {
#define IWFPM_CASE(s) \
    case s:                                                \
        if constexpr (s <= MAXS) pencil_conv<s, R>(base, es, vp); \
        break;
        IWFPM_EXTENTS(IWFPM_CASE)
#undef IWFPM_CASE
        default: break;
    }
}

// all pencils of one axis of an LDS tile: pencil p starts at
// (p / es) * es * S + p % es and steps by es
template <int SIGN, typename R, int MAXS>
__device__ __forceinline__ void run_axis(cplx<R>* lds, int S, int npencil, int es) {
    for (int p = threadIdx.x; p < npencil; p += blockDim.x) {
        int hi = p / es, lo = p - hi * es;
        dispatch_fft<SIGN, R, MAXS>(S, lds + hi * es * S + lo, es);
    }
}

// ---------------------------------------------------------------------------
// index maps (Sec. 3.2)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int pmod(int a, int m) {
    int r = a % m;
    return r < 0 ? r + m : r;
}

// window-order position r (within one vector) -> grid-order position
__device__ __forceinline__ int vec_to_grid(const DevGeom& g, const int* __restrict__ slice_a, int r) {
    int s = (int)(r / g.nkI);
    int q = r - s * (int)g.nkI;
    int out = s * (int)g.nkI;
    for (int j = g.d - 1; j >= 0; --j) {
        int ax = g.n - g.d + j;
        int E = g.ext[ax];
        int pj = q % E;
        q /= E;
        out += pmod(pj + slice_a[s * g.d + j], E) * (int)g.stride[ax];
    }
    return out;
}

// grid-order position -> window-order position
__device__ __forceinline__ int grid_to_vec(const DevGeom& g, const int* __restrict__ slice_a, int r) {
    int s = (int)(r / g.nkI);
    int q = r - s * (int)g.nkI;
    int out = s * (int)g.nkI;
    for (int j = g.d - 1; j >= 0; --j) {
        int ax = g.n - g.d + j;
        int E = g.ext[ax];
        int kj = q % E;
        q /= E;
        out += pmod(kj - slice_a[s * g.d + j], E) * (int)g.stride[ax];
    }
    return out;
}

// Lambda at grid position r: k_II from the slice (eq:inverse2), k_I = a +
// ((k* - a) mod 2K) (eq:inverse3 written with the slice's lower window end a),
// then 1/2 |2 pi P_II k_II + 2 pi P_I k_I|^2 in float64.
__device__ __forceinline__ double kinetic_at(const DevGeom& g, const int* __restrict__ slice_a,
                                             const double* __restrict__ slice_g, int r) {
    int s = (int)(r / g.nkI);
    int q = r - s * (int)g.nkI;
    double kI[kMaxAxes];
    for (int j = g.d - 1; j >= 0; --j) {
        int ax = g.n - g.d + j;
        int E = g.ext[ax];
        int ks = q % E;
        q /= E;
        int a = slice_a[s * g.d + j];
        kI[j] = (double)(a + pmod(ks - a, E));
    }
    double tot = 0.0;
    for (int j = 0; j < g.d; ++j) {
        double v = slice_g[s * g.d + j];
        for (int i = 0; i < g.d; ++i) v += g.P1[j * g.d + i] * kI[i];
        tot += v * v;
    }
    return 0.5 * tot;
}

template <typename R>
__device__ __forceinline__ const R* vtab_of(const DevTabs& t);
template <>
__device__ __forceinline__ const float* vtab_of<float>(const DevTabs& t) { return t.vtab32; }
template <>
__device__ __forceinline__ const double* vtab_of<double>(const DevTabs& t) { return t.vtab64; }
template <typename R>
__device__ __forceinline__ const R* vgrid_of(const DevTabs& t);
template <>
__device__ __forceinline__ const float* vgrid_of<float>(const DevTabs& t) { return t.vgrid32; }
template <>
__device__ __forceinline__ const double* vgrid_of<double>(const DevTabs& t) { return t.vgrid64; }

// sum of the per-axis potential tables at grid position r, axis `skip` left out
template <typename R>
__device__ __forceinline__ R vsum_except(const DevGeom& g, const R* __restrict__ vtab, int r, int skip) {
    R acc = R(0);
    for (int ax = 0; ax < g.n; ++ax) {
        if (ax == skip) continue;
        int l = (int)((r / g.stride[ax]) % g.ext[ax]);
        acc += vtab[g.voff[ax] + l];
    }
    return acc;
}

template <typename R>
__device__ __forceinline__ VPencil<R> make_vpencil(const DevGeom& g, const DevTabs& t, int ax, int gbase) {
    VPencil<R> vp;
    vp.gbase = gbase;
    vp.gstep = (int)g.stride[ax];
    if (g.vmode == 1) {
        vp.vgrid = vgrid_of<R>(t);
        vp.vaxis = nullptr;
        vp.vb = R(0);
    } else {
        vp.vgrid = nullptr;
        const R* vt = vtab_of<R>(t);
        vp.vaxis = vt + g.voff[ax];
        vp.vb = vsum_except<R>(g, vt, gbase, ax);
    }
    return vp;
}

__device__ __forceinline__ int remap_block(int bid, int nblocks, int on) {
    // Workgroups are dealt round-robin over the 8 XCDs; give XCD x a
    // contiguous run of tiles so neighbouring tiles share its L2.
    if (!on || nblocks < 16) return bid;
    int per = nblocks / 8, rem = nblocks - per * 8;
    int xcd = bid & 7, local = bid >> 3;
    if (local < per) return xcd * per + local;
    (void)rem;
    return bid;  // the ragged tail keeps its order
}

// ---------------------------------------------------------------------------
// fused schedule: one vector per workgroup
// ---------------------------------------------------------------------------

template <typename R, int MAXS>
__global__ void __launch_bounds__(256) k_fused(DevGeom g, DevTabs t, const double2* __restrict__ psi,
                                               double2* __restrict__ hpsi) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem);
    const int N = (int)g.N;
    const long long off = (long long)blockIdx.x * g.N;
    const double2* __restrict__ x = psi + off;
    double2* __restrict__ y = hpsi + off;

    for (int e = threadIdx.x; e < N; e += blockDim.x) {
        int gp = g.order ? vec_to_grid(g, t.slice_a, e) : e;
        double2 v = x[e];
        tile[gp] = cplx<R>{R(v.x), R(v.y)};
    }
    __syncthreads();
    for (int ax = 0; ax < g.n - 1; ++ax) {
        run_axis<+1, R, MAXS>(tile, g.ext[ax], N / g.ext[ax], (int)g.stride[ax]);
        __syncthreads();
    }
    {
        const int ax = g.n - 1;
        const int S = g.ext[ax], es = (int)g.stride[ax], np = N / S;
        for (int p = threadIdx.x; p < np; p += blockDim.x) {
            int hi = p / es, lo = p - hi * es;
            int base = hi * es * S + lo;
            VPencil<R> vp = make_vpencil<R>(g, t, ax, base);
            dispatch_conv<R, MAXS>(S, tile + base, es, vp);
        }
        __syncthreads();
    }
    for (int ax = g.n - 2; ax >= 0; --ax) {
        run_axis<-1, R, MAXS>(tile, g.ext[ax], N / g.ext[ax], (int)g.stride[ax]);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < N; e += blockDim.x) {
        int vp = g.order ? grid_to_vec(g, t.slice_a, e) : e;
        double lam = kinetic_at(g, t.slice_a, t.slice_g, e);
        double2 xv = x[vp];
        cplx<R> c = tile[e];
        y[vp] = make_double2(lam * xv.x + (double)c.x, lam * xv.y + (double)c.y);
    }
}

// ---------------------------------------------------------------------------
// three-pass schedule
// ---------------------------------------------------------------------------

// pass 1: gather (window order) + inverse DFT along the trailing axes
template <typename R, int MAXS>
__global__ void __launch_bounds__(256) k_pass1(DevGeom g, DevTabs t, PassDesc pd, const double2* __restrict__ psi,
                                               cplx<R>* __restrict__ ws, long long nslab) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem);
    const int G = pd.slabs_per_wg;
    const int sin_ = (int)pd.s_in;
    const int bid = remap_block(blockIdx.x, gridDim.x, pd.xcd_remap);
    const long long slab0 = (long long)bid * G;
    const int nsl = (int)min((long long)G, nslab - slab0);
    const int nload = nsl * sin_;
    const long long gbase = slab0 * sin_;

    for (int e = threadIdx.x; e < G * sin_; e += blockDim.x) {
        if (e < nload) {
            long long gi = gbase + e;
            double2 v = psi[gi];
            int lo = e;
            if (g.order) {
                long long vec = gi / g.N;
                int r = (int)(gi - vec * g.N);
                lo = (int)(vec * g.N + vec_to_grid(g, t.slice_a, r) - gbase);
            }
            tile[lo] = cplx<R>{R(v.x), R(v.y)};
        } else {
            tile[e] = cplx<R>{R(0), R(0)};
        }
    }
    __syncthreads();
    for (int ax = pd.split; ax < g.n; ++ax) {
        run_axis<+1, R, MAXS>(tile, g.ext[ax], G * sin_ / g.ext[ax], (int)g.stride[ax]);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < nload; e += blockDim.x) ws[gbase + e] = tile[e];
}

// pass 2: inverse DFT along the leading axes, x V, forward DFT, on a tile of
// `tile` consecutive columns of one vector
template <typename R, int MAXS>
__global__ void __launch_bounds__(256) k_pass2(DevGeom g, DevTabs t, PassDesc pd, cplx<R>* __restrict__ ws) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem);
    const int T = pd.tile;
    const int sin_ = (int)pd.s_in, sout = (int)pd.s_out;
    const int ntile = (sin_ + T - 1) / T;
    const int bid = remap_block(blockIdx.x, gridDim.x, pd.xcd_remap);
    const int vec = bid / ntile;
    const int c0 = (bid - vec * ntile) * T;
    const int tw = min(T, sin_ - c0);
    cplx<R>* __restrict__ w = ws + (long long)vec * g.N;

    for (int e = threadIdx.x; e < sout * T; e += blockDim.x) {
        int o = e / T, tt = e - o * T;
        tile[e] = tt < tw ? w[(long long)o * sin_ + c0 + tt] : cplx<R>{R(0), R(0)};
    }
    __syncthreads();
    const int split = pd.split;
    for (int ax = 0; ax < split - 1; ++ax) {
        int es = (int)(g.stride[ax] / sin_) * T;
        run_axis<+1, R, MAXS>(tile, g.ext[ax], sout * T / g.ext[ax], es);
        __syncthreads();
    }
    {
        const int ax = split - 1;
        const int S = g.ext[ax];
        const int es = (int)(g.stride[ax] / sin_) * T;
        const int np = sout * T / S;
        for (int p = threadIdx.x; p < np; p += blockDim.x) {
            int hi = p / es, lo = p - hi * es;
            int base = hi * es * S + lo;
            int tt = base % T;
            int ob = base / T;
            int gb = ob * sin_ + c0 + min(tt, tw - 1);
            VPencil<R> vp = make_vpencil<R>(g, t, ax, gb);
            dispatch_conv<R, MAXS>(S, tile + base, es, vp);
        }
        __syncthreads();
    }
    for (int ax = split - 2; ax >= 0; --ax) {
        int es = (int)(g.stride[ax] / sin_) * T;
        run_axis<-1, R, MAXS>(tile, g.ext[ax], sout * T / g.ext[ax], es);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < sout * T; e += blockDim.x) {
        int o = e / T, tt = e - o * T;
        if (tt < tw) w[(long long)o * sin_ + c0 + tt] = tile[e];
    }
}

// pass 3: forward DFT along the trailing axes + kinetic term + scatter
template <typename R, int MAXS>
__global__ void __launch_bounds__(256) k_pass3(DevGeom g, DevTabs t, PassDesc pd, const double2* __restrict__ psi,
                                               const cplx<R>* __restrict__ ws, double2* __restrict__ hpsi,
                                               long long nslab) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem);
    const int G = pd.slabs_per_wg;
    const int sin_ = (int)pd.s_in;
    const int bid = remap_block(blockIdx.x, gridDim.x, pd.xcd_remap);
    const long long slab0 = (long long)bid * G;
    const int nsl = (int)min((long long)G, nslab - slab0);
    const int nload = nsl * sin_;
    const long long gbase = slab0 * sin_;

    for (int e = threadIdx.x; e < G * sin_; e += blockDim.x)
        tile[e] = e < nload ? ws[gbase + e] : cplx<R>{R(0), R(0)};
    __syncthreads();
    for (int ax = g.n - 1; ax >= pd.split; --ax) {
        run_axis<-1, R, MAXS>(tile, g.ext[ax], G * sin_ / g.ext[ax], (int)g.stride[ax]);
        __syncthreads();
    }
    for (int e = threadIdx.x; e < nload; e += blockDim.x) {
        long long gi = gbase + e;
        long long vec = gi / g.N;
        int r = (int)(gi - vec * g.N);
        long long vi = g.order ? vec * g.N + grid_to_vec(g, t.slice_a, r) : gi;
        double lam = kinetic_at(g, t.slice_a, t.slice_g, r);
        double2 xv = psi[vi];
        cplx<R> c = tile[e];
        hpsi[vi] = make_double2(lam * xv.x + (double)c.x, lam * xv.y + (double)c.y);
    }
}

}  // namespace iwfpm
