// eigfun.hip - the eigenfunction in physical space (eq:int, the interpolant
// I_{K,L} of Alg. 1's last step):
//
//     u(xi) = sum over the window of U_k exp(i 2 pi (P k) . xi)
//
// on a tensor observation grid xi_j = o_j + h_j i_j.  The exponential of the
// sum over the d coordinates is the product of d per-axis exponentials, so
// with E_j[k][i] = exp(i 2 pi (P k)_j xi_j(i)) the grid values are one dense
// complex contraction over the N window points:
//
//     u[m][c] = sum_k A[k][m] B[k][c],
//     A[k][m] = U_k prod_{j < d-1} E_j[k][i_j(m)],   B[k][c] = E_{d-1}[k][c],
//
// m running over the first d-1 axes (row-major) and c over the last.  The
// per-axis tables are built for a chunk of window points at a time; the
// contraction runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64, four real
// products per complex one), split over the window points into slices whose
// partial grids are summed in a fixed order, so results do not depend on the
// launch shape's timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/iwfpm.h"
#include "plan.hpp"

namespace iwfpm {
namespace {

typedef double ef_d4 __attribute__((ext_vector_type(4)));

constexpr int kEfTile = 64;        // output rows and columns per workgroup
constexpr int kEfDepth = 4;        // 4-point groups of the contraction in flight per wave
constexpr int kEfMaxDim = 6;

__device__ __forceinline__ double2 ef_cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// table of one axis for window points [p0, p0 + np): out[p * n + i] =
// exp(i 2 pi f[p0 + p] (o + h i)), times U[p0 + p] when U is given.  The phase
// is reduced to one turn before the sine and cosine.
__global__ void k_ef_table(const double* __restrict__ f, const double2* __restrict__ U, long long p0, long long np,
                           int n, double o, double h, double2* __restrict__ out) {
    const long long total = np * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const long long p = e / n;
        const int i = (int)(e - p * n);
        double t = f[p0 + p] * (o + h * (double)i);
        t -= rint(t);
        double s, c;
        sincospi(2.0 * t, &s, &c);
        double2 v = make_double2(c, s);
        if (U) v = ef_cmul(v, U[p0 + p]);
        out[e] = v;
    }
}

struct EfGemm {
    int d;                         // physical dimensions
    long long M;                   // rows: points of the first d-1 axes (1 when d = 1)
    int nc;                        // columns: points of the last axis
    int na[kEfMaxDim];             // the first d-1 axes' lengths
    long long aoff[kEfMaxDim];     // their tables (rows of na[j] entries)
    long long boff;                // the last axis' table (rows of nc entries)
    const double2* U;              // d = 1: the A operand is U[p0 + p] itself
    long long p0;                  // first window point of the chunk
    long long np;                  // window points in the chunk
    long long ps;                  // window points per slice (a multiple of 4)
    int tiles_m, tiles_c;
    int accumulate;                // add to the output (a later chunk) instead of overwriting
};

__device__ __forceinline__ void ef_load(const double2* __restrict__ tab, const EfGemm& g, long long pp, long long pe,
                                        bool mok, const long long (&arow)[kEfMaxDim], int cb, int li, double2& a,
                                        double2 (&b)[4]) {
    const bool pok = pp < pe;
    a = make_double2(0.0, 0.0);
    if (pok && mok) {
        if (g.d == 1) {
            a = g.U[g.p0 + pp];
        } else {
            a = tab[g.aoff[0] + pp * g.na[0] + arow[0]];
            for (int j = 1; j < g.d - 1; ++j) a = ef_cmul(a, tab[g.aoff[j] + pp * g.na[j] + arow[j]]);
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = cb + 16 * t + li;
        b[t] = (pok && c < g.nc) ? tab[g.boff + pp * g.nc + c] : make_double2(0.0, 0.0);
    }
}

// One workgroup: a 64 x 64 tile of the grid (four waves of 16 rows, each
// wave four 16-column MFMA tiles) over one slice of the window points.  Lane
// l holds A[l%16][l/16] and B[l/16][l%16] of each 16 x 4 x 16 product and
// ends with D[l/16 + 4v][l%16]; the contraction index runs over groups of 4
// window points, lane l taking point 4g + l/16.
__global__ void __launch_bounds__(256) k_ef_gemm(const double2* __restrict__ tab, EfGemm g,
                                                 double2* __restrict__ partial, double2* __restrict__ out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    long long b = blockIdx.x;
    const int tc = (int)(b % g.tiles_c);
    b /= g.tiles_c;
    const int tm = (int)(b % g.tiles_m);
    const long long s = b / g.tiles_m;
    const long long m = (long long)tm * kEfTile + 16 * wave + li;
    const bool mok = m < g.M;
    long long arow[kEfMaxDim] = {0, 0, 0, 0, 0, 0};
    if (g.d > 1) {
        long long r = mok ? m : 0;
        for (int j = g.d - 2; j >= 0; --j) {
            arow[j] = r % g.na[j];
            r /= g.na[j];
        }
    }
    const int cb = tc * kEfTile;
    const long long pb = s * g.ps, pe = min(g.np, pb + g.ps);
    ef_d4 accr[4], acci[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        accr[t] = ef_d4{0.0, 0.0, 0.0, 0.0};
        acci[t] = ef_d4{0.0, 0.0, 0.0, 0.0};
    }
    constexpr int D = kEfDepth;
    double2 ab[D], bb[D][4];
#pragma unroll
    for (int u = 0; u < D; ++u) ef_load(tab, g, pb + 4 * u + lk, pe, mok, arow, cb, li, ab[u], bb[u]);
    for (long long p = pb; p < pe; p += 4 * D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const double2 a = ab[u];
            double2 bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) bv[t] = bb[u][t];
            ef_load(tab, g, p + 4 * (u + D) + lk, pe, mok, arow, cb, li, ab[u], bb[u]);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bv[t].x, accr[t], 0, 0, 0);
                acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bv[t].y, acci[t], 0, 0, 0);
                accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, bv[t].y, accr[t], 0, 0, 0);
                acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, bv[t].x, acci[t], 0, 0, 0);
            }
        }
    }
    const long long total = g.M * g.nc;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = cb + 16 * t + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const long long row = (long long)tm * kEfTile + 16 * wave + lk + 4 * v;
            if (row < g.M && c < g.nc) {
                const long long e = row * g.nc + c;
                double2 val = make_double2(accr[t][v], acci[t][v]);
                if (out) {  // one slice: this lane owns the element
                    if (g.accumulate) {
                        const double2 o = out[e];
                        val = make_double2(o.x + val.x, o.y + val.y);
                    }
                    out[e] = val;
                } else {
                    partial[s * total + e] = val;
                }
            }
        }
    }
}

// out[e] = (accumulate ? out[e] : 0) + sum over the slices, in slice order
__global__ void k_ef_reduce(const double2* __restrict__ partial, int S, long long total, int accumulate,
                            double2* __restrict__ out) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        double2 acc = accumulate ? out[e] : make_double2(0.0, 0.0);
        for (int s = 0; s < S; ++s) {
            const double2 v = partial[(long long)s * total + e];
            acc.x += v.x;
            acc.y += v.y;
        }
        out[e] = acc;
    }
}

__global__ void k_ef_zero(long long total, double2* __restrict__ out) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x)
        out[e] = make_double2(0.0, 0.0);
}

constexpr size_t kEfTableBudget = (size_t)256 << 20;    // bytes of per-axis tables per chunk
constexpr size_t kEfPartialBudget = (size_t)512 << 20;  // bytes of slice partials

// the frequencies (P k)_j of every window point, axis-major (d x N), in the
// plan's vector order; built on the host from the labels once per plan
int ensure_freq(iwfpm_plan_s* p, hipStream_t st) {
    const long long N = p->geom.N;
    const size_t bytes = (size_t)p->d * (size_t)N * sizeof(double);
    if (p->d_ef_freq.ptr && p->d_ef_freq.bytes >= bytes) return IWFPM_OK;
    std::vector<double> f((size_t)p->d * (size_t)N);
    std::vector<int> k(p->n);
    for (long long gp = 0; gp < N; ++gp) {
        host_label(p, gp, k.data());
        const long long vp = host_grid_to_vec(p, gp);
        for (int j = 0; j < p->d; ++j) {
            double acc = 0.0;
            for (int l = 0; l < p->n; ++l) acc += p->P[(size_t)j * p->n + l] * (double)k[l];
            f[(size_t)j * N + vp] = acc;
        }
    }
    dev_free(p->d_ef_freq);
    if (int rc = dev_alloc(p->d_ef_freq, bytes)) return rc;
    if (hipMemcpyAsync(p->d_ef_freq.ptr, f.data(), bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    return IWFPM_OK;
}

int grid_blocks(long long work) { return (int)std::max(1LL, std::min(4096LL, (work + 255) / 256)); }

}  // namespace
}  // namespace iwfpm

using namespace iwfpm;

extern "C" int iwfpm_eigenfunction(iwfpm_plan_t p, const void* u, const double* origin, const double* step,
                                   const int* npts, void* out, void* stream) {
    if (!p || !u || !origin || !step || !npts || !out) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    const int d = p->d;
    if (d < 1 || d > kEfMaxDim) return IWFPM_ERR_ARG;
    long long total = 1;
    for (int j = 0; j < d; ++j) {
        if (npts[j] < 1 || !std::isfinite(origin[j]) || !std::isfinite(step[j])) return IWFPM_ERR_ARG;
        total *= npts[j];
        if (total > (1LL << 36)) return IWFPM_ERR_ARG;  // keeps tiles x slices within one launch
    }
    DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    const long long N = p->geom.N;
    if (int rc = ensure_freq(p, st)) return rc;

    EfGemm g{};
    g.d = d;
    g.M = 1;
    for (int j = 0; j + 1 < d; ++j) {
        g.na[j] = npts[j];
        g.M *= npts[j];
    }
    g.nc = npts[d - 1];
    g.U = (const double2*)u;
    g.tiles_m = (int)((g.M + kEfTile - 1) / kEfTile);
    g.tiles_c = (g.nc + kEfTile - 1) / kEfTile;
    const long long tiles = (long long)g.tiles_m * g.tiles_c;
    // table entries per window point: the A-side axes (none when d = 1) and the last axis
    long long row = g.nc;
    for (int j = 0; j + 1 < d; ++j) row += g.na[j];
    long long np = (long long)(kEfTableBudget / (sizeof(double2) * (size_t)row));
    np = std::max(4LL, np - np % 4);
    np = std::min(np, ((N + 3) / 4) * 4);
    // slices: enough workgroups for the chip, at least 64 window points each,
    // partials within their budget (one slice writes the output directly)
    long long S = std::max(1LL, std::min((2048 + tiles - 1) / tiles, 64LL));
    S = std::min(S, std::max(1LL, np / 64));
    S = std::min(S, std::max(1LL, (long long)(kEfPartialBudget / (sizeof(double2) * (size_t)total))));
    const size_t tab_bytes = sizeof(double2) * (size_t)np * (size_t)row;
    const size_t part_bytes = S > 1 ? sizeof(double2) * (size_t)S * (size_t)total : 0;
    if (!p->d_ef_ws.ptr || p->d_ef_ws.bytes < tab_bytes + part_bytes) {
        if (hipStreamSynchronize(st) != hipSuccess) return IWFPM_ERR_DEVICE;
        dev_free(p->d_ef_ws);
        if (int rc = dev_alloc(p->d_ef_ws, tab_bytes + part_bytes)) return rc;
    }
    double2* tab = (double2*)p->d_ef_ws.ptr;
    double2* part = S > 1 ? tab + (size_t)np * (size_t)row : nullptr;
    double2* o = (double2*)out;
    const double* f = (const double*)p->d_ef_freq.ptr;

    if (N == 0) {
        k_ef_zero<<<grid_blocks(total), 256, 0, st>>>(total, o);
        return hipGetLastError() == hipSuccess ? IWFPM_OK : IWFPM_ERR_DEVICE;
    }
    for (long long p0 = 0; p0 < N; p0 += np) {
        const long long cnt = std::min(np, N - p0);
        g.p0 = p0;
        g.np = cnt;
        // table offsets within the chunk buffer
        long long off = 0;
        for (int j = 0; j + 1 < d; ++j) {
            g.aoff[j] = off;
            k_ef_table<<<grid_blocks(cnt * g.na[j]), 256, 0, st>>>(f + (size_t)j * N, j == 0 ? g.U : nullptr, p0, cnt,
                                                                 g.na[j], origin[j], step[j], tab + off);
            off += cnt * g.na[j];
        }
        g.boff = off;
        k_ef_table<<<grid_blocks(cnt * g.nc), 256, 0, st>>>(f + (size_t)(d - 1) * N, nullptr, p0, cnt, g.nc,
                                                          origin[d - 1], step[d - 1], tab + off);
        long long Sc = std::min(S, std::max(1LL, cnt / 64));
        g.ps = (((cnt + Sc - 1) / Sc) + 3) / 4 * 4;
        Sc = (cnt + g.ps - 1) / g.ps;
        g.accumulate = p0 > 0;
        k_ef_gemm<<<dim3((unsigned)(tiles * Sc)), 256, 0, st>>>(tab, g, part, Sc == 1 ? o : nullptr);
        if (Sc > 1) k_ef_reduce<<<grid_blocks(total), 256, 0, st>>>(part, (int)Sc, total, g.accumulate, o);
        if (hipGetLastError() != hipSuccess) return IWFPM_ERR_DEVICE;
    }
    return IWFPM_OK;
}
