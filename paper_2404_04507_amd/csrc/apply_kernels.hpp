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
// tile between axes.  Slab tiles pad their last (contiguous) axis to an odd
// pitch so that the pencils along it, one per lane, hit distinct banks.  The
// per-element index work of the gather / scatter and of the kinetic term is
// hoisted into a per-row table (a row = one line along the last axis): within
// a row the true label along the last axis only wraps once, so each element
// costs a compare and a few fused multiply-adds.

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
#define IWFPM_CASE(s)                                              \
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
#define IWFPM_CASE(s)                                             \
    case s:                                                      \
        if constexpr (s <= MAXS) pencil_conv<s, R>(base, es, vp); \
        break;
        IWFPM_EXTENTS(IWFPM_CASE)
#undef IWFPM_CASE
        default: break;
    }
}

// Division by a divisor d that is the same for the whole workgroup, for
// dividends and divisors below 2^16 (every position inside an LDS tile: a
// tile holds at most 20,480 float entries).  The float quotient a * rcp(d),
// with rcp(d) within one ulp of 1/d, is within a/d * 2^-22 < 2^-6 of a/d, so
// its truncation is off by at most one, and one integer correction step
// makes it exact (checked for every d < 2^16 with reciprocals one ulp off
// either way).  The integer division it replaces takes some thirty
// instructions; this takes about six.
struct Div16 {
    int d;
    float inv;
    __device__ __forceinline__ explicit Div16(int dd) : d(dd), inv(__builtin_amdgcn_rcpf((float)dd)) {}
    __device__ __forceinline__ int div(int a) const {
        int q = (int)((float)a * inv);
        const int r = a - q * d;
        q += (r >= d) - (r < 0);
        return q;
    }
};

// Pencil p of an axis with extent S and logical element stride es starts at
// the logical offset (p / es) * es * S + p % es.  A logical offset L maps to
// (L / sl) * sp + L % sl in a tile whose rows of sl elements are padded to a
// pitch sp; a pencil either stays inside one row (es < sl) or steps by whole
// rows (es a multiple of sl).
__device__ __forceinline__ int phys(int L, RowGeom rg, const Div16& dsl) {
    const int r = dsl.div(L);
    return r * rg.sp + (L - r * rg.sl);
}

// ---------------------------------------------------------------------------
// long axes: S = f_0 f_1 ... f_{m-1} points, more than one register pencil
// ---------------------------------------------------------------------------
//
// The inverse DFT of length S runs in m in-place stages over the LDS tile.
// Stage i works on blocks of B_i = f_i ... f_{m-1} consecutive points (block
// b at offset b B_i); within a block it takes the f_i points at stride
// s_i = B_i / f_i starting at r < s_i, applies an f_i-point DFT, multiplies
// output k by e^{2 pi i r k / B_i} (not in the last stage, where s_i = 1) and
// writes the results back to the same positions.  This is the decimation in
// frequency of the DFT into its factors: afterwards position
// p = p_0 s_0 + p_1 s_1 + ... + p_{m-1} holds the transform at
// l = p_0 + f_0 (p_1 + f_1 (p_2 + ...)), the digit-reversed order of p.
// The forward DFT is the adjoint of the inverse one: the same stages in
// reverse order, each with the conjugate twiddles applied before an f_i-point
// DFT of the opposite sign, which returns natural order.  Between the two the
// axis stays in digit order; only the potential, which is indexed by l, has
// to know (unperm_pos).

template <typename R>
__device__ __forceinline__ const cplx<R>* tw_of(const DevTabs& t, const DevGeom& g, int ax);
template <>
__device__ __forceinline__ const cplx<float>* tw_of<float>(const DevTabs& t, const DevGeom& g, int ax) {
    return reinterpret_cast<const cplx<float>*>(t.tw32) + g.twoff[ax];
}
template <>
__device__ __forceinline__ const cplx<double>* tw_of<double>(const DevTabs& t, const DevGeom& g, int ax) {
    return reinterpret_cast<const cplx<double>*>(t.tw64) + g.twoff[ax];
}

// digit order -> natural order along a long axis (position c -> index l)
__device__ __forceinline__ int long_axis_perm(const DevGeom& g, int ax, int c) {
    int l = 0, mult = 1, B = g.ext[ax];
    for (int i = 0; i < g.nfac[ax]; ++i) {
        const int f = g.fac[ax][i];
        const int st = B / f;
        const int k = c / st;
        c -= k * st;
        l += mult * k;
        mult *= f;
        B = st;
    }
    return l;
}

// storage position of the grid (long axes in digit order) -> grid position
__device__ __forceinline__ int unperm_pos(const DevGeom& g, int pos) {
    int out = pos;
    for (int ax = 0; ax < g.n; ++ax) {
        if (g.nfac[ax] <= 1) continue;
        const int c = (pos / g.stride[ax]) % g.ext[ax];
        out += (long_axis_perm(g, ax, c) - c) * g.stride[ax];
    }
    return out;
}

// npencil pencils of S points at logical element stride es, each one DFT in
// registers
template <int SIGN, typename R, int MAXS>
__device__ __forceinline__ void run_axis(cplx<R>* lds, int S, int npencil, int es, RowGeom rg) {
    const int pes = es < rg.sl ? es : (es / rg.sl) * rg.sp;
    const Div16 des(es), dsl(rg.sl);
    for (int p = threadIdx.x; p < npencil; p += blockDim.x) {
        const int hi = des.div(p), lo = p - hi * es;
        dispatch_fft<SIGN, R, MAXS>(S, lds + phys(hi * es * S + lo, rg, dsl), pes);
    }
}

// The twiddles of one stage of a long axis, on the pencils of run_axis with
// the same arguments and the same pencil-to-thread assignment (so every
// thread touches only what it transforms itself, and no barrier is needed
// between the two): entry k of the pencil with offset r = (p mod es) / es_tw
// in its block is multiplied by tw[r k mult] (conjugated for SIGN < 0).  A
// loop of its own, so that run_axis keeps the bare pencil loop.
template <int SIGN, typename R>
__device__ __forceinline__ void twiddle_axis(cplx<R>* lds, int S, int npencil, int es, RowGeom rg,
                                             const cplx<R>* __restrict__ tw, int es_tw, int mult) {
    const int pes = es < rg.sl ? es : (es / rg.sl) * rg.sp;
    const Div16 des(es), dsl(rg.sl), dtw(es_tw);
    for (int p = threadIdx.x; p < npencil; p += blockDim.x) {
        const int hi = des.div(p), lo = p - hi * es;
        const int tstep = dtw.div(lo) * mult;
        if (!tstep) continue;
        cplx<R>* base = lds + phys(hi * es * S + lo, rg, dsl);
        for (int k = 1; k < S; ++k) {
            const cplx<R> w = tw[k * tstep];
            cplx<R>& v = base[k * pes];
            if (SIGN > 0) v = cplx<R>{v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x};
            else v = cplx<R>{v.x * w.x + v.y * w.y, v.y * w.x - v.x * w.y};
        }
    }
}

// The transform along axis ax of every pencil of the tile (npencil pencils at
// logical element stride es).  A long axis runs its stages as sweeps of
// run_axis (and twiddle_axis): stage i has sub-pencils of f_i points at stride (B_i / f_i) es,
// and sub-pencil (block b, offset r) of the axis' pencil (hi, lo) starts at
// hi es S + lo + (b B_i + r) es = hi' (B_i / f_i) es f_i + lo' with
// lo' = r es + lo, i.e. exactly where run_axis puts pencil (hi', lo').
template <int SIGN, typename R, int MAXS>
__device__ __forceinline__ void run_axis_any(const DevGeom& g, const DevTabs& t, int ax, cplx<R>* lds, int npencil,
                                             int es, RowGeom rg) {
    const int S = g.ext[ax], m = g.nfac[ax];
    for (int st = 0; st < m; ++st) {
        // one call site of run_axis, so that the kernel inlines the register
        // pencils once; a one-stage axis does none of the stage arithmetic
        int f = S, np = npencil, esf = es, mult = 0;
        const cplx<R>* tw = nullptr;
        if (m > 1) {
            const int i = SIGN > 0 ? st : m - 1 - st;
            int B = S;
            for (int j = 0; j < i; ++j) B /= g.fac[ax][j];
            f = g.fac[ax][i];
            np = npencil * (S / f);
            esf = (B / f) * es;
            mult = S / B;
            if (i < m - 1) tw = tw_of<R>(t, g, ax);
        }
        if (SIGN < 0 && tw) twiddle_axis<SIGN, R>(lds, f, np, esf, rg, tw, es, mult);
        run_axis<SIGN, R, MAXS>(lds, f, np, esf, rg);
        if (SIGN > 0 && tw) twiddle_axis<SIGN, R>(lds, f, np, esf, rg, tw, es, mult);
        if (st + 1 < m) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// index maps (Sec. 3.2)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int pmod(int a, int m) {
    int r = a % m;
    return r < 0 ? r + m : r;
}

// Per-row data of the kinetic term and of the window order, for the row whose
// first element sits at grid position r0 (a multiple of the last extent):
//   B_j    = 2 pi (P_II k_II)_j + sum_{i < d-1} (2 pi P_I)_{j i} k_i     (j < d)
//   alast  = lower window end of the last k_I axis in this slice
//   amod   = alast mod ext_last
//   vrow   = vector position of the row's first element in window order
//            (minus the rotation of the last axis), or r0 in grid order
// With them, the element in column c of the row has the last true label
// k_last = alast + ((c - amod) mod ext_last) (eq:inverse3 in floor form) and
// Lambda = 1/2 sum_j (B_j + (2 pi P_I)_{j, d-1} k_last)^2.
struct RowTable {
    double* B;   // rows x d
    int* alast;
    int* amod;
    int* vrow;
};

__device__ __forceinline__ RowTable row_table_at(unsigned char* base, int rows, int d) {
    RowTable t;
    t.B = reinterpret_cast<double*>(base);
    t.alast = reinterpret_cast<int*>(t.B + (size_t)rows * d);
    t.amod = t.alast + rows;
    t.vrow = t.amod + rows;
    return t;
}

__device__ __forceinline__ void row_entry(const DevGeom& g, const DevTabs& t, int r0, RowTable tab, int row) {
    const int d = g.d, n = g.n;
    const int s = r0 / g.nkI;
    int q = r0 - s * g.nkI;
    const int* a = t.slice_a + s * d;
    const double* gg = t.slice_g + s * d;
    double kI[kMaxAxes];
    int vrow = s * g.nkI;
    q /= g.ext[n - 1];  // the row starts at column 0 of the last axis
    for (int j = d - 2; j >= 0; --j) {
        int ax = n - d + j;
        int E = g.ext[ax];
        int ks = q % E;
        q /= E;
        int pj = pmod(ks - a[j], E);
        kI[j] = (double)(a[j] + pj);
        vrow += (g.order ? pj : ks) * g.stride[ax];
    }
    for (int j = 0; j < d; ++j) {
        double b = gg[j];
        for (int i = 0; i < d - 1; ++i) b += g.P1[j * d + i] * kI[i];
        tab.B[row * d + j] = b;
    }
    const int El = g.ext[n - 1];
    tab.alast[row] = a[d - 1];
    tab.amod[row] = pmod(a[d - 1], El);
    tab.vrow[row] = vrow;
}

// kinetic term and vector position of column c of a row (see RowTable)
__device__ __forceinline__ double row_kinetic(const DevGeom& g, const RowTable& tab, int row, int c, int* vpos) {
    const int d = g.d;
    const int El = g.ext[g.n - 1];
    int pl = c - tab.amod[row];
    pl += pl < 0 ? El : 0;
    const double kl = (double)(tab.alast[row] + pl);
    double lam = 0.0;
    for (int j = 0; j < d; ++j) {
        double v = tab.B[row * d + j] + g.P1[j * d + d - 1] * kl;
        lam += v * v;
    }
    *vpos = tab.vrow[row] + (g.order ? pl : c);
    return 0.5 * lam;
}

// window-order position r (within one vector) -> grid-order position
__device__ __forceinline__ int vec_to_grid(const DevGeom& g, const int* __restrict__ slice_a, int r) {
    int s = r / g.nkI;
    int q = r - s * g.nkI;
    int out = s * g.nkI;
    for (int j = g.d - 1; j >= 0; --j) {
        int ax = g.n - g.d + j;
        int E = g.ext[ax];
        int pj = q % E;
        q /= E;
        out += pmod(pj + slice_a[s * g.d + j], E) * g.stride[ax];
    }
    return out;
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
        int l = (r / g.stride[ax]) % g.ext[ax];
        acc += vtab[g.voff[ax] + l];
    }
    return acc;
}

template <typename R>
__device__ __forceinline__ VPencil<R> make_vpencil(const DevGeom& g, const DevTabs& t, int ax, int gbase) {
    VPencil<R> vp;
    gbase = unperm_pos(g, gbase);  // the other axes may be long and in digit order
    vp.gbase = gbase;
    vp.gstep = g.stride[ax];
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

// V / N at a storage position of the grid (long axes in digit order)
template <typename R>
__device__ __forceinline__ R v_at_storage(const DevGeom& g, const DevTabs& t, int pos) {
    const int gp = unperm_pos(g, pos);
    if (g.vmode == 1) return vgrid_of<R>(t)[gp];
    return vsum_except<R>(g, vtab_of<R>(t), gp, -1);
}

__device__ __forceinline__ int remap_block(int bid, int nblocks, int on) {
    // Workgroups are dealt round-robin over the 8 XCDs; give XCD x a
    // contiguous run of tiles so neighbouring tiles share its L2.
    if (!on || nblocks < 16) return bid;
    int per = nblocks / 8;
    int xcd = bid & 7, local = bid >> 3;
    if (local < per) return xcd * per + local;
    return bid;  // the ragged tail keeps its order
}

// independent global loads each thread keeps in flight in the tile copies
constexpr int kBatch = 8;

// two adjacent complex entries, moved as one access
template <typename R>
struct alignas(16) CPair {
    cplx<R> a, b;
};

// element iterator over a tile of `rows` rows of length sl: thread-strided,
// with row / column updated incrementally (no division per element)
struct RowIter {
    int e, row, col, drow, dcol, sl;
    __device__ __forceinline__ RowIter(int start, int step, int sl_) : e(start), sl(sl_) {
        row = start / sl_;
        col = start - row * sl_;
        drow = step / sl_;
        dcol = step - drow * sl_;
    }
    __device__ __forceinline__ void next(int step) {
        e += step;
        row += drow;
        col += dcol;
        if (col >= sl) {
            col -= sl;
            ++row;
        }
    }
};

// load `count` vector-order elements starting at vector position v0 into a
// grid-order LDS tile (padded rows); in window order the rows are gathered
template <typename R>
__device__ __forceinline__ void load_gather(const DevGeom& g, const DevTabs& t, const double2* __restrict__ x,
                                            int v0, int count, cplx<R>* tile, RowGeom rg, int* rowmap) {
    const int nt = blockDim.x;
    if (g.order) {
        // rowmap[rv] = (grid row within the tile) * sp, and the rotation of the last axis
        const int rows = count / rg.sl;
        for (int rv = threadIdx.x; rv < rows; rv += nt) {
            int gp = vec_to_grid(g, t.slice_a, v0 + rv * rg.sl);  // element 0 of this vector row
            int grow = (gp - v0) / rg.sl;
            rowmap[2 * rv] = grow * rg.sp;
            rowmap[2 * rv + 1] = gp - v0 - grow * rg.sl;  // its column = a_last mod sl
        }
        __syncthreads();
        for (RowIter it(threadIdx.x, nt, rg.sl); it.e < count;) {
            double2 v[kBatch];
            RowIter j = it;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                v[u] = j.e < count ? x[v0 + j.e] : make_double2(0.0, 0.0);
                j.next(nt);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (it.e < count) {
                    int c = it.col + rowmap[2 * it.row + 1];
                    c -= c >= rg.sl ? rg.sl : 0;
                    tile[rowmap[2 * it.row] + c] = cplx<R>{R(v[u].x), R(v[u].y)};
                }
                it.next(nt);
            }
        }
    } else {
        for (RowIter it(threadIdx.x, nt, rg.sl); it.e < count;) {
            double2 v[kBatch];
            RowIter j = it;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                v[u] = j.e < count ? x[v0 + j.e] : make_double2(0.0, 0.0);
                j.next(nt);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (it.e < count) tile[it.row * rg.sp + it.col] = cplx<R>{R(v[u].x), R(v[u].y)};
                it.next(nt);
            }
        }
    }
}

// Nontemporal access for data the apply touches for the last time: the
// intermediate grid when the last pass reads it, and H psi when it is
// written.  Neither needs to stay in the caches, and marking them so leaves
// the room to psi and to the grid still in use by the other passes (pass 3
// 77 -> 71 us and pass 1 60 -> 51 us on the 589,824-point, 16-vector block).
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cplx<float> nt_load(const cplx<float>* p) {
    nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
    return {v.x, v.y};
}
__device__ __forceinline__ cplx<double> nt_load(const cplx<double>* p) {
    nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    return {v.x, v.y};
}

// copy `count` grid-order elements of the intermediate grid (its last read:
// nontemporal) into a padded tile, kBatch independent loads in flight per thread
template <typename R>
__device__ __forceinline__ void load_tile(const cplx<R>* __restrict__ w, int count, cplx<R>* tile, RowGeom rg) {
    const int nt = blockDim.x;
    if constexpr (sizeof(cplx<R>) == 8) {
        // float entries: adjacent pairs (rows of even length, 16-byte aligned
        // start) as one 16-byte load, stored to LDS as two entries
        if ((rg.sl & 1) == 0 && (count & 1) == 0 && (reinterpret_cast<uintptr_t>(w) & 15) == 0) {
            const int count2 = count >> 1;
            const nt_f4* w4 = reinterpret_cast<const nt_f4*>(w);
            for (RowIter it(threadIdx.x, nt, rg.sl >> 1); it.e < count2;) {
                nt_f4 v[kBatch];
                RowIter j = it;
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    v[u] = j.e < count2 ? __builtin_nontemporal_load(w4 + j.e) : nt_f4{0.f, 0.f, 0.f, 0.f};
                    j.next(nt);
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    if (it.e < count2) {
                        cplx<R>* d = tile + it.row * rg.sp + 2 * it.col;
                        d[0] = cplx<R>{v[u].x, v[u].y};
                        d[1] = cplx<R>{v[u].z, v[u].w};
                    }
                    it.next(nt);
                }
            }
            return;
        }
    }
    for (RowIter it(threadIdx.x, nt, rg.sl); it.e < count;) {
        cplx<R> v[kBatch];
        RowIter j = it;
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            v[u] = j.e < count ? nt_load(&w[j.e]) : cplx<R>{R(0), R(0)};
            j.next(nt);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (it.e < count) tile[it.row * rg.sp + it.col] = v[u];
            it.next(nt);
        }
    }
}

template <typename R>
__device__ __forceinline__ void store_tile(cplx<R>* __restrict__ w, int count, const cplx<R>* tile, RowGeom rg) {
    const int nt = blockDim.x;
    if constexpr (sizeof(cplx<R>) == 8) {
        // float entries: adjacent pairs as one 16-byte store (as in load_tile)
        if ((rg.sl & 1) == 0 && (count & 1) == 0 && (reinterpret_cast<uintptr_t>(w) & 15) == 0) {
            float4* w4 = reinterpret_cast<float4*>(w);
            for (RowIter it(threadIdx.x, nt, rg.sl >> 1); it.e < (count >> 1); it.next(nt)) {
                const cplx<R>* s = tile + it.row * rg.sp + 2 * it.col;
                w4[it.e] = make_float4(s[0].x, s[0].y, s[1].x, s[1].y);
            }
            return;
        }
    }
    for (RowIter it(threadIdx.x, nt, rg.sl); it.e < count; it.next(nt)) w[it.e] = tile[it.row * rg.sp + it.col];
}

// kinetic term + scatter for `count` grid-order elements starting at grid
// position r0 of one vector: y[v] = Lambda x[v] + tile
template <typename R>
__device__ __forceinline__ void kinetic_scatter(const DevGeom& g, const DevTabs& t, const double2* __restrict__ x,
                                                double2* __restrict__ y, int r0, int count, const cplx<R>* tile,
                                                RowGeom rg, RowTable tab) {
    const int nt = blockDim.x;
    const int rows = count / rg.sl;
    for (int r = threadIdx.x; r < rows; r += nt) row_entry(g, t, r0 + r * rg.sl, tab, r);
    __syncthreads();
    for (RowIter it(threadIdx.x, nt, rg.sl); it.e < count;) {
        int vpos[kBatch];
        double lam[kBatch];
        double2 xv[kBatch];
        RowIter j = it;
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (j.e < count) {
                lam[u] = row_kinetic(g, tab, j.row, j.col, &vpos[u]);
                xv[u] = g.kin ? x[vpos[u]] : make_double2(0.0, 0.0);
            }
            j.next(nt);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (it.e < count) {
                cplx<R> c = tile[it.row * rg.sp + it.col];
                __builtin_nontemporal_store(nt_d2{lam[u] * xv[u].x + (double)c.x, lam[u] * xv[u].y + (double)c.y},
                                            reinterpret_cast<nt_d2*>(y + vpos[u]));
            }
            it.next(nt);
        }
    }
}

// ---------------------------------------------------------------------------
// fused schedule: one vector per workgroup
// ---------------------------------------------------------------------------

template <typename R, int MAXS>
__device__ __forceinline__ void fused_body(const DevGeom& g, const DevTabs& t, RowGeom rg,
                                           const double2* __restrict__ psi, double2* __restrict__ hpsi, int vecid,
                                           unsigned char* smem) {
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem);
    const int N = g.N;
    const int rows = N / rg.sl;
    unsigned char* extra = smem + (size_t)rows * rg.sp * sizeof(cplx<R>);
    const long long off = (long long)vecid * N;
    const double2* __restrict__ x = psi + off;
    double2* __restrict__ y = hpsi + off;

    load_gather<R>(g, t, x, 0, N, tile, rg, reinterpret_cast<int*>(extra));
    __syncthreads();
    // A long last axis takes its inverse stages with the other axes, then the
    // potential at every point, then its forward stages; a short one keeps
    // inverse, potential and forward DFT of each line in registers.
    const bool long_last = g.nfac[g.n - 1] > 1;
    const int n_inv = long_last ? g.n : g.n - 1;
    for (int ax = 0; ax < n_inv; ++ax) {
        run_axis_any<+1, R, MAXS>(g, t, ax, tile, N / g.ext[ax], g.stride[ax], rg);
        __syncthreads();
    }
    if (long_last) {
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl); it.e < N; it.next(blockDim.x)) {
            cplx<R>& c = tile[it.row * rg.sp + it.col];
            c = cscale(c, v_at_storage<R>(g, t, it.e));
        }
    } else {
        const int S = rg.sl;
        for (int p = threadIdx.x; p < rows; p += blockDim.x) {
            VPencil<R> vp = make_vpencil<R>(g, t, g.n - 1, p * S);
            dispatch_conv<R, MAXS>(S, tile + p * rg.sp, 1, vp);
        }
    }
    __syncthreads();
    for (int ax = n_inv - 1; ax >= 0; --ax) {
        run_axis_any<-1, R, MAXS>(g, t, ax, tile, N / g.ext[ax], g.stride[ax], rg);
        __syncthreads();
    }
    kinetic_scatter<R>(g, t, x, y, 0, N, tile, rg, row_table_at(extra, rows, g.d));
}

template <typename R, int MAXS>
__global__ void __launch_bounds__(256) k_fused(DevGeom g, DevTabs t, RowGeom rg, const double2* __restrict__ psi,
                                               double2* __restrict__ hpsi) {
    extern __shared__ __align__(16) unsigned char smem[];
    fused_body<R, MAXS>(g, t, rg, psi, hpsi, blockIdx.x, smem);
}

// ---------------------------------------------------------------------------
// three-pass schedule.  Passes 1 and 3 give each workgroup up to
// slabs_per_wg consecutive slabs of one vector.
// ---------------------------------------------------------------------------

// pass 1: gather (window order) + inverse DFT along the trailing axes
template <typename R, int MAXS>
__device__ __forceinline__ void pass1_body(const DevGeom& g, const DevTabs& t, const PassDesc& pd, RowGeom rg,
                                           const double2* __restrict__ psi, cplx<R>* __restrict__ ws, int bid_raw,
                                           int nblocks, unsigned char* smem) {
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem);
    const int G = pd.slabs_per_wg, sin_ = pd.s_in;
    const int bpv = (pd.s_out + G - 1) / G;
    const int bid = remap_block(bid_raw, nblocks, pd.xcd_remap);
    const int vec = bid / bpv;
    const int slab0 = (bid - vec * bpv) * G;
    const int nsl = min(G, pd.s_out - slab0);
    const int count = nsl * sin_;
    const int r0 = slab0 * sin_;
    const long long off = (long long)vec * g.N;
    unsigned char* extra = smem + (size_t)(G * sin_ / rg.sl) * rg.sp * sizeof(cplx<R>);

    load_gather<R>(g, t, psi + off, r0, count, tile, rg, reinterpret_cast<int*>(extra));
    __syncthreads();
    for (int ax = pd.split; ax < g.n; ++ax) {
        run_axis_any<+1, R, MAXS>(g, t, ax, tile, count / g.ext[ax], g.stride[ax], rg);
        __syncthreads();
    }
    store_tile<R>(ws + off + r0, count, tile, rg);
}

template <typename R, int MAXS>
__global__ void __launch_bounds__(256, sizeof(R) == 8 ? 2 : 1) k_pass1(DevGeom g, DevTabs t, PassDesc pd, RowGeom rg,
                                               const double2* __restrict__ psi, cplx<R>* __restrict__ ws) {
    extern __shared__ __align__(16) unsigned char smem[];
    pass1_body<R, MAXS>(g, t, pd, rg, psi, ws, blockIdx.x, gridDim.x, smem);
}

// The middle pass's outermost axis (axis 0, one register pencil) between
// global memory and the LDS tile: its inverse DFT runs on values loaded from
// global memory before they first reach the tile, its forward DFT on values
// read from the tile for the last time, which go to global memory from the
// registers.  This takes the place of the tile's copy-in and copy-out sweeps
// and of their barriers.  A thread takes the pencils of two adjacent columns
// (16-byte accesses); the pair's element j sits at global offset gofs + j gstep
// and at tile offset lofs + j lstep.
template <int S, int SIGN, typename R>
__device__ __forceinline__ void p2_axis0_pair(cplx<R>* __restrict__ w, cplx<R>* tile, int gofs, int gstep, int lofs,
                                              int lstep) {
    cplx<R> a[S], b[S];
    if constexpr (SIGN > 0) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const CPair<R> v = *reinterpret_cast<const CPair<R>*>(w + gofs + j * gstep);
            a[j] = v.a;
            b[j] = v.b;
        }
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const CPair<R> v = *reinterpret_cast<const CPair<R>*>(tile + lofs + j * lstep);
            a[j] = v.a;
            b[j] = v.b;
        }
    }
    fft_inplace<S, SIGN>(a);
    fft_inplace<S, SIGN>(b);
    if constexpr (SIGN > 0) {
#pragma unroll
        for (int j = 0; j < S; ++j) *reinterpret_cast<CPair<R>*>(tile + lofs + j * lstep) = CPair<R>{a[j], b[j]};
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) *reinterpret_cast<CPair<R>*>(w + gofs + j * gstep) = CPair<R>{a[j], b[j]};
    }
}

// the same with one column per thread (8-byte accesses for float32), for
// tiles with fewer column pairs than the workgroup has threads
template <int S, int SIGN, typename R>
__device__ __forceinline__ void p2_axis0_one(cplx<R>* __restrict__ w, cplx<R>* tile, int gofs, int gstep, int lofs,
                                             int lstep) {
    cplx<R> a[S];
    if constexpr (SIGN > 0) {
#pragma unroll
        for (int j = 0; j < S; ++j) a[j] = w[gofs + j * gstep];
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) a[j] = tile[lofs + j * lstep];
    }
    fft_inplace<S, SIGN>(a);
    if constexpr (SIGN > 0) {
#pragma unroll
        for (int j = 0; j < S; ++j) tile[lofs + j * lstep] = a[j];
    } else {
#pragma unroll
        for (int j = 0; j < S; ++j) w[gofs + j * gstep] = a[j];
    }
}

// longest axis 0 taken this way: two pencils of it in registers take 128 VGPRs
template <typename R>
constexpr int kAxis0Max = 256 / (int)sizeof(cplx<R>);

// every pencil pair of axis 0 of the tile: count elements in rows of sl = El T
// (T even), axis 0 of extent S0 stepping R0 = count / (S0 sl) tile rows
template <int SIGN, typename R, int MAXS>
__device__ __forceinline__ void p2_axis0(int S0, cplx<R>* __restrict__ w, cplx<R>* tile, int count, int El, int lgT,
                                         int sin_, RowGeom rg) {
    const int np2 = count / S0 / 2;
    const int R0 = count / (S0 * rg.sl);
    const int T = 1 << lgT;
    const Div16 dsl(rg.sl);
    if (np2 < (int)blockDim.x) {
        // fewer pairs than threads: one column per thread keeps them all busy
        for (int p = threadIdx.x; p < 2 * np2; p += blockDim.x) {
            const int row0 = dsl.div(p), col = p - row0 * rg.sl;
            const int gofs = (row0 * El + (col >> lgT)) * sin_ + (col & (T - 1));
            const int gstep = R0 * El * sin_;
            const int lofs = row0 * rg.sp + col, lstep = R0 * rg.sp;
            switch (S0) {
#define IWFPM_CASE(s)                                                                 \
    case s:                                                                          \
        if constexpr (s <= MAXS && s <= kAxis0Max<R>) p2_axis0_one<s, SIGN, R>(w, tile, gofs, gstep, lofs, lstep); \
        break;
                IWFPM_EXTENTS(IWFPM_CASE)
#undef IWFPM_CASE
                default: break;
            }
        }
        return;
    }
    for (int q = threadIdx.x; q < np2; q += blockDim.x) {
        const int row0 = dsl.div(2 * q), col = 2 * q - row0 * rg.sl;
        const int gofs = (row0 * El + (col >> lgT)) * sin_ + (col & (T - 1));
        const int gstep = R0 * El * sin_;
        const int lofs = row0 * rg.sp + col, lstep = R0 * rg.sp;
        switch (S0) {
#define IWFPM_CASE(s)                                                                  \
    case s:                                                                           \
        if constexpr (s <= MAXS && s <= kAxis0Max<R>) p2_axis0_pair<s, SIGN, R>(w, tile, gofs, gstep, lofs, lstep); \
        break;
            IWFPM_EXTENTS(IWFPM_CASE)
#undef IWFPM_CASE
            default: break;
        }
    }
}

// Per-axis potential tables (vmode 0) in the middle pass: the sum over the
// axes other than the convolution axis (the last leading one) splits into a
// part fixed by the tile row (the other leading axes) and a part fixed by the
// column (the trailing axes).  Row e of the tile starts at leading position
// e El (convolution axis at 0); cc is a column of the trailing block.
template <typename R>
__device__ __forceinline__ R p2_row_sum(const DevGeom& g, const R* vt, int split, int sin_, int e) {
    const int o = e * g.ext[split - 1];
    R acc = R(0);
    for (int a = 0; a < split - 1; ++a) {
        int c = (o / (g.stride[a] / sin_)) % g.ext[a];
        if (g.nfac[a] > 1) c = long_axis_perm(g, a, c);
        acc += vt[g.voff[a] + c];
    }
    return acc;
}
template <typename R>
__device__ __forceinline__ R p2_col_sum(const DevGeom& g, const R* vt, int split, int cc) {
    R acc = R(0);
    for (int a = split; a < g.n; ++a) {
        int c = (cc / g.stride[a]) % g.ext[a];
        if (g.nfac[a] > 1) c = long_axis_perm(g, a, c);
        acc += vt[g.voff[a] + c];
    }
    return acc;
}

// inverse DFT, x V, forward DFT along the convolution axis (El points at
// element stride T = 2^lgT) of every pencil of the tile, with the row and
// column sums tabulated (a pencil reads two entries instead of decomposing
// its grid position) and vaxis the convolution axis' own table
template <typename R, int MAXS>
__device__ __forceinline__ void p2_conv_tables(cplx<R>* tile, RowGeom rg, int count, int El, int lgT, const R* vrow,
                                               const R* vcol, const R* vaxis) {
    const int T = 1 << lgT;
    const int np = count / El;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const int hi = p >> lgT, lo = p & (T - 1);  // hi: row, lo: column
        VPencil<R> vp;
        vp.vgrid = nullptr;
        vp.vaxis = vaxis;
        vp.vb = vrow[hi] + vcol[lo];
        vp.gbase = 0;
        vp.gstep = 0;
        dispatch_conv<R, MAXS>(El, tile + hi * rg.sp + lo, T, vp);
    }
}

// pass 2: inverse DFT along the leading axes, x V, forward DFT, on a tile of
// `tile` consecutive columns of one vector.  The LDS tile is [outer][column];
// its rows (one line of the last leading axis times the columns) are padded
// by `tile` entries, which spreads the lanes of the pencils along that axis
// over distinct banks.
template <typename R, int MAXS>
__device__ __forceinline__ void pass2_body(const DevGeom& g, const DevTabs& t, const PassDesc& pd,
                                           cplx<R>* __restrict__ ws, int bid_raw, int nblocks, unsigned char* smem) {
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem);
    const int T = pd.tile, lgT = __ffs(T) - 1;
    const int sin_ = pd.s_in, sout = pd.s_out;
    const int ntile = (sin_ + T - 1) / T;
    const int bid = remap_block(bid_raw, nblocks, pd.xcd_remap);
    const int vec = bid / ntile;
    const int c0 = (bid - vec * ntile) * T;
    const int tw = min(T, sin_ - c0);
    cplx<R>* __restrict__ w = ws + (long long)vec * g.N + c0;
    const int split = pd.split;
    const int El = g.ext[split - 1];
    const RowGeom rg{El << lgT, (El + 1) << lgT};
    const int count = sout << lgT;

    // logical element e = row * (El T) + col: outer index o = row El + col / T, column col % T.
    // With an even, whole tile the columns come in pairs that are adjacent in
    // memory and in LDS (all extents are even, so the pairs stay aligned):
    // they move as one access each, twice the bytes in flight per load.
    const bool pairs = (T & 1) == 0 && tw == T;
    // then axis 0, when it is not the convolution axis and is one register
    // pencil, moves straight between global memory and the tile (p2_axis0)
    const bool fuse0 = pairs && split >= 2 && g.nfac[0] == 1 && g.ext[0] <= kAxis0Max<R>;
    if (fuse0) {
        p2_axis0<+1, R, MAXS>(g.ext[0], w, tile, count, El, lgT, sin_, rg);
    } else if (pairs) {
        const int count2 = count >> 1;
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl >> 1); it.e < count2;) {
            CPair<R> v[kBatch];
            RowIter j = it;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int col = 2 * j.col;
                const int o = j.row * El + (col >> lgT), tt = col & (T - 1);
                v[u] = j.e < count2 ? *reinterpret_cast<const CPair<R>*>(w + o * sin_ + tt) : CPair<R>{};
                j.next(blockDim.x);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (it.e < count2) *reinterpret_cast<CPair<R>*>(tile + it.row * rg.sp + 2 * it.col) = v[u];
                it.next(blockDim.x);
            }
        }
    } else {
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl); it.e < count;) {
            cplx<R> v[kBatch];
            RowIter j = it;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                int o = j.row * El + (j.col >> lgT), tt = j.col & (T - 1);
                v[u] = (j.e < count && tt < tw) ? w[o * sin_ + tt] : cplx<R>{R(0), R(0)};
                j.next(blockDim.x);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (it.e < count) tile[it.row * rg.sp + it.col] = v[u];
                it.next(blockDim.x);
            }
        }
    }
    __syncthreads();
    // as in the fused kernel: a long last leading axis takes its inverse
    // stages with the other leading axes, then the potential at every point of
    // the tile, then its forward stages
    const bool long_last = g.nfac[split - 1] > 1;
    const int n_inv = long_last ? split : split - 1;
    for (int ax = fuse0 ? 1 : 0; ax < n_inv; ++ax) {
        int es = (g.stride[ax] / sin_) << lgT;
        run_axis_any<+1, R, MAXS>(g, t, ax, tile, count / g.ext[ax], es, rg);
        __syncthreads();
    }
    if (long_last) {
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl); it.e < count; it.next(blockDim.x)) {
            const int i = it.col >> lgT, tt = it.col & (T - 1);
            if (tt < tw) {
                cplx<R>& c = tile[it.row * rg.sp + it.col];
                c = cscale(c, v_at_storage<R>(g, t, (it.row * El + i) * sin_ + c0 + tt));
            }
        }
    } else if (g.vmode == 0) {
        // per-axis potential tables: row and column sums tabulated per tile
        // (after the tile)
        const int nrow = count / rg.sl;
        R* vrow = reinterpret_cast<R*>(smem + (size_t)nrow * rg.sp * sizeof(cplx<R>));
        R* vcol = vrow + nrow;
        const R* vt = vtab_of<R>(t);
        for (int e = threadIdx.x; e < nrow + T; e += blockDim.x)
            vrow[e] = e < nrow ? p2_row_sum<R>(g, vt, split, sin_, e)
                               : p2_col_sum<R>(g, vt, split, c0 + min(e - nrow, tw - 1));
        __syncthreads();
        p2_conv_tables<R, MAXS>(tile, rg, count, El, lgT, vrow, vcol, vt + g.voff[split - 1]);
    } else {
        const int ax = split - 1;
        const int S = El;
        const int es = T;
        const int np = count / S;
        for (int p = threadIdx.x; p < np; p += blockDim.x) {
            int hi = p >> lgT, lo = p & (T - 1);  // hi: row, lo: column
            int gb = hi * El * sin_ + c0 + min(lo, tw - 1);
            VPencil<R> vp = make_vpencil<R>(g, t, ax, gb);
            dispatch_conv<R, MAXS>(S, tile + hi * rg.sp + lo, es, vp);
        }
    }
    __syncthreads();
    for (int ax = n_inv - 1; ax >= (fuse0 ? 1 : 0); --ax) {
        int es = (g.stride[ax] / sin_) << lgT;
        run_axis_any<-1, R, MAXS>(g, t, ax, tile, count / g.ext[ax], es, rg);
        __syncthreads();
    }
    if (fuse0) {
        p2_axis0<-1, R, MAXS>(g.ext[0], w, tile, count, El, lgT, sin_, rg);
    } else if (pairs) {
        const int count2 = count >> 1;
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl >> 1); it.e < count2; it.next(blockDim.x)) {
            const int col = 2 * it.col;
            const int o = it.row * El + (col >> lgT), tt = col & (T - 1);
            *reinterpret_cast<CPair<R>*>(w + o * sin_ + tt) =
                *reinterpret_cast<const CPair<R>*>(tile + it.row * rg.sp + col);
        }
    } else {
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl); it.e < count; it.next(blockDim.x)) {
            int o = it.row * El + (it.col >> lgT), tt = it.col & (T - 1);
            if (tt < tw) w[o * sin_ + tt] = tile[it.row * rg.sp + it.col];
        }
    }
}

// pass M: the DFT (SIGN) along axes [a, b) alone, a = split_mid and b = split,
// on a tile of `tile_mid` consecutive columns (the index over the axes from b
// on) of one outer index (the axes before a) of one vector.  The LDS tile has
// pass 2's layout with the axes [a, b) in place of the leading block.
template <int SIGN, typename R, int MAXS>
__device__ __forceinline__ void passm_body(const DevGeom& g, const DevTabs& t, const PassDesc& pd,
                                           cplx<R>* __restrict__ ws, int bid_raw, int nblocks,
                                           unsigned char* smem) {
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem);
    const int a = pd.split_mid, b = pd.split;
    const int T = pd.tile_mid, lgT = __ffs(T) - 1;
    const int cols = pd.s_in;                       // product of the extents from b on
    const int mid = g.stride[a - 1] / cols;         // product of the extents in [a, b)
    const int outer = g.N / (mid * cols);           // product of the extents before a
    const int ntile = (cols + T - 1) / T;
    const int bid = remap_block(bid_raw, nblocks, pd.xcd_remap);
    const int vec = bid / (outer * ntile);
    const int rem = bid - vec * outer * ntile;
    const int o = rem / ntile;
    const int c0 = (rem - o * ntile) * T;
    const int tw = min(T, cols - c0);
    cplx<R>* __restrict__ w = ws + (long long)vec * g.N + (long long)o * mid * cols + c0;
    const int El = g.ext[b - 1];
    const RowGeom rg{El << lgT, (El + 1) << lgT};
    const int count = mid << lgT;
    // element e = row * (El T) + col: index within [a, b) = row El + col / T,
    // column col % T; an even, whole tile moves adjacent column pairs as one
    // access (as in the middle pass)
    const bool pairs = (T & 1) == 0 && tw == T;
    if (pairs) {
        const int count2 = count >> 1;
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl >> 1); it.e < count2;) {
            CPair<R> v[kBatch];
            RowIter j = it;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int col = 2 * j.col;
                const int q = j.row * El + (col >> lgT), tt = col & (T - 1);
                v[u] = j.e < count2 ? *reinterpret_cast<const CPair<R>*>(w + q * cols + tt) : CPair<R>{};
                j.next(blockDim.x);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (it.e < count2) *reinterpret_cast<CPair<R>*>(tile + it.row * rg.sp + 2 * it.col) = v[u];
                it.next(blockDim.x);
            }
        }
    } else {
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl); it.e < count;) {
            cplx<R> v[kBatch];
            RowIter j = it;
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int q = j.row * El + (j.col >> lgT), tt = j.col & (T - 1);
                v[u] = (j.e < count && tt < tw) ? w[q * cols + tt] : cplx<R>{R(0), R(0)};
                j.next(blockDim.x);
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                if (it.e < count) tile[it.row * rg.sp + it.col] = v[u];
                it.next(blockDim.x);
            }
        }
    }
    __syncthreads();
    for (int ax = a; ax < b; ++ax) {
        const int es = (g.stride[ax] / cols) << lgT;
        run_axis_any<SIGN, R, MAXS>(g, t, ax, tile, count / g.ext[ax], es, rg);
        __syncthreads();
    }
    if (pairs) {
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl >> 1); it.e < (count >> 1); it.next(blockDim.x)) {
            const int col = 2 * it.col;
            const int q = it.row * El + (col >> lgT), tt = col & (T - 1);
            *reinterpret_cast<CPair<R>*>(w + q * cols + tt) =
                *reinterpret_cast<const CPair<R>*>(tile + it.row * rg.sp + col);
        }
    } else {
        for (RowIter it(threadIdx.x, blockDim.x, rg.sl); it.e < count; it.next(blockDim.x)) {
            const int q = it.row * El + (it.col >> lgT), tt = it.col & (T - 1);
            if (tt < tw) w[q * cols + tt] = tile[it.row * rg.sp + it.col];
        }
    }
}

// Largest workgroup of the middle pass and of the further pass.  Their LDS
// tile is large (up to 160 KB), so often one workgroup holds a CU alone, and
// then only a large workgroup gives the CU enough waves to keep its loads in
// flight.  That case is a leading block of many short axes (16^3 on the 6D
// grid: 1,024 pencils per axis in a 4-column tile); 1024 threads cap a thread
// at 128 VGPRs and 512 at 256, which 16-point pencils fit without spilling
// (float32: 1024, float64: 512).  Longer pencils keep 256: their blocks have
// fewer pencils than that per axis, and a kernel bound for more threads than
// it can use measured slower.
template <typename R, int MAXS>
constexpr int wide_pass_threads() {
    return MAXS <= 16 ? (sizeof(R) == 4 ? 1024 : 512) : 256;
}

template <int SIGN, typename R, int MAXS>
__global__ void __launch_bounds__((wide_pass_threads<R, MAXS>()))
    k_passm(DevGeom g, DevTabs t, PassDesc pd, cplx<R>* __restrict__ ws) {
    extern __shared__ __align__(16) unsigned char smem[];
    passm_body<SIGN, R, MAXS>(g, t, pd, ws, blockIdx.x, gridDim.x, smem);
}

template <typename R, int MAXS>
__global__ void __launch_bounds__((wide_pass_threads<R, MAXS>()))
    k_pass2(DevGeom g, DevTabs t, PassDesc pd, cplx<R>* __restrict__ ws) {
    extern __shared__ __align__(16) unsigned char smem[];
    pass2_body<R, MAXS>(g, t, pd, ws, blockIdx.x, gridDim.x, smem);
}

// pass 3: forward DFT along the trailing axes + kinetic term + scatter
template <typename R, int MAXS>
__device__ __forceinline__ void pass3_body(const DevGeom& g, const DevTabs& t, const PassDesc& pd, RowGeom rg,
                                           const double2* __restrict__ psi, const cplx<R>* __restrict__ ws,
                                           double2* __restrict__ hpsi, int bid_raw, int nblocks,
                                           unsigned char* smem) {
    cplx<R>* tile = reinterpret_cast<cplx<R>*>(smem);
    const int G = pd.slabs_per_wg, sin_ = pd.s_in;
    const int bpv = (pd.s_out + G - 1) / G;
    const int bid = remap_block(bid_raw, nblocks, pd.xcd_remap);
    const int vec = bid / bpv;
    const int slab0 = (bid - vec * bpv) * G;
    const int nsl = min(G, pd.s_out - slab0);
    const int count = nsl * sin_;
    const int r0 = slab0 * sin_;
    const long long off = (long long)vec * g.N;
    unsigned char* extra = smem + (size_t)(G * sin_ / rg.sl) * rg.sp * sizeof(cplx<R>);

    load_tile<R>(ws + off + r0, count, tile, rg);
    __syncthreads();
    for (int ax = g.n - 1; ax >= pd.split; --ax) {
        run_axis_any<-1, R, MAXS>(g, t, ax, tile, count / g.ext[ax], g.stride[ax], rg);
        __syncthreads();
    }
    kinetic_scatter<R>(g, t, psi + off, hpsi + off, r0, count, tile, rg,
                       row_table_at(extra, G * sin_ / rg.sl, g.d));
}

template <typename R, int MAXS>
__global__ void __launch_bounds__(256, sizeof(R) == 8 ? 2 : 1) k_pass3(DevGeom g, DevTabs t, PassDesc pd, RowGeom rg,
                                               const double2* __restrict__ psi, const cplx<R>* __restrict__ ws,
                                               double2* __restrict__ hpsi) {
    extern __shared__ __align__(16) unsigned char smem[];
    pass3_body<R, MAXS>(g, t, pd, rg, psi, ws, hpsi, blockIdx.x, gridDim.x, smem);
}

// ---------------------------------------------------------------------------
// ragged batches: one persistent launch per pass walks a work table of many
// plans (e.g. a sweep of couplings whose windows differ).  Work items of
// instance i are [start[i], start[i+1]); every workgroup strides over the
// items, so the grid size is independent of the batch and a captured graph
// of the launches stays valid while the table in device memory changes.
// ---------------------------------------------------------------------------

struct BatchItem {
    DevGeom g;
    DevTabs t;
    PassDesc pd;
    RowGeom rg;
    const double2* psi;
    double2* hpsi;
    void* ws;
    int fused;
    int start[3];  // first work item of this instance in passes 1, 2, 3 (fused: pass 1 = vectors)
};

struct BatchHead {
    int B;
    int total[3];  // work items per pass
};

__device__ __forceinline__ int find_item(const BatchItem* __restrict__ items, int B, int pass, int w) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (items[mid].start[pass] <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename R, int MAXS>
__global__ void __launch_bounds__(256) k_batch_pass(const BatchHead* __restrict__ head,
                                                    const BatchItem* __restrict__ items, int pass) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int B = head->B, total = head->total[pass];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int i = find_item(items, B, pass, w);
        const BatchItem& it = items[i];
        const int end = i + 1 < B ? items[i + 1].start[pass] : total;
        const int local = w - it.start[pass], nb = end - it.start[pass];
        __syncthreads();  // the previous item's LDS tile is no longer read
        if (it.fused) {
            if (pass == 0) fused_body<R, MAXS>(it.g, it.t, it.rg, it.psi, it.hpsi, local, smem);
        } else if (pass == 0) {
            pass1_body<R, MAXS>(it.g, it.t, it.pd, it.rg, it.psi, reinterpret_cast<cplx<R>*>(it.ws), local, nb, smem);
        } else if (pass == 1) {
            pass2_body<R, MAXS>(it.g, it.t, it.pd, reinterpret_cast<cplx<R>*>(it.ws), local, nb, smem);
        } else {
            pass3_body<R, MAXS>(it.g, it.t, it.pd, it.rg, it.psi, reinterpret_cast<const cplx<R>*>(it.ws), it.hpsi,
                                local, nb, smem);
        }
    }
}

}  // namespace iwfpm
