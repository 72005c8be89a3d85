// plan.cpp - iwfpm_plan and the geometry / potential set-up (Alg. 1 steps 1-2).
//
// Built without floating-point contraction so that the sheared offsets
// q = Q k_II are formed exactly as written (ties at integers stay ties).

#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>

#include "apply_launch.hpp"
#include "sizes.hpp"

using namespace iwfpm;

namespace iwfpm {

static const double kTwoPi = 6.283185307179586476925286766559;

static bool pencil_compiled(int e) {
    switch (e) {
#define IWFPM_CASE(s) \
    case s: return true;
        IWFPM_EXTENTS(IWFPM_CASE)
#undef IWFPM_CASE
        default: return false;
    }
}

// Stages of an axis transform: one register pencil when the extent is
// compiled, else the most balanced split into two (then three) compiled
// pencil sizes > 1, the largest stage last; 0 stages if there is none.
int axis_factors(int e, int* fac) {
    if (e < 1) return 0;
    if (pencil_compiled(e)) {
        fac[0] = e;
        return 1;
    }
    int best = 0, bmax = 1 << 30;
    for (int a = 2; a * a <= e; ++a) {
        if (e % a || !pencil_compiled(a) || !pencil_compiled(e / a)) continue;
        if (e / a < bmax) {
            bmax = e / a;
            fac[0] = a;
            fac[1] = e / a;
            best = 2;
        }
    }
    if (best) return best;
    for (int a = 2; a * a * a <= e; ++a) {
        if (e % a || !pencil_compiled(a)) continue;
        const int r = e / a;
        for (int b = a; b * b <= r; ++b) {
            if (r % b || !pencil_compiled(b) || !pencil_compiled(r / b)) continue;
            if (r / b < bmax) {
                bmax = r / b;
                fac[0] = a;
                fac[1] = b;
                fac[2] = r / b;
                best = 3;
            }
        }
    }
    return best;
}

static bool extent_supported(int e) {
    int f[kMaxFactors];
    return axis_factors(e, f) > 0;
}

static int extent_class(int e) { return e <= 16 ? 16 : (e <= 32 ? 32 : 64); }
int extent_class_of(int e) { return extent_class(e); }

// the register pencils an axis needs: its largest stage
int axis_class(const DevGeom& g, int ax) {
    int m = 0;
    for (int i = 0; i < g.nfac[ax]; ++i) m = std::max(m, g.fac[ax][i]);
    return extent_class(m);
}

// largest workgroup of the middle and further passes for an extent class
// (the device rule of wide_pass_threads)
static int wide_pass_threads(int prec, int maxs) { return maxs <= 16 ? (prec == 1 ? 1024 : 512) : 256; }

// pencils (or, for long axes, sub-pencils of the most numerous stage) that
// one transform along axis ax of a tile of `count` points has to process
static int axis_items(const DevGeom& g, int ax, long long count) {
    int mn = g.ext[ax];
    for (int i = 0; i < g.nfac[ax]; ++i) mn = std::min(mn, g.fac[ax][i]);
    return (int)(count / mn);
}

int dev_alloc(DeviceBuf& b, size_t bytes) {
    dev_free(b);
    if (bytes == 0) return IWFPM_OK;
    if (hipMalloc(&b.ptr, bytes) != hipSuccess) {
        b.ptr = nullptr;
        (void)hipGetLastError();
        return IWFPM_ERR_ALLOC;
    }
    b.bytes = bytes;
    return IWFPM_OK;
}

void dev_free(DeviceBuf& b) {
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
}

// Solve P_I X = P_II by Gaussian elimination with partial pivoting (Sec. 3.1).
static int solve_Q(int d, int n, const double* P, std::vector<double>& Q) {
    const int m = n - d;
    std::vector<double> A(d * d), B(d * m);
    double scale = 0.0;
    for (int i = 0; i < d; ++i) {
        for (int j = 0; j < d; ++j) A[i * d + j] = P[i * n + j];
        for (int j = 0; j < m; ++j) B[i * m + j] = P[i * n + d + j];
        for (int j = 0; j < n; ++j) scale = std::max(scale, std::fabs(P[i * n + j]));
    }
    if (!(scale > 0.0)) return IWFPM_ERR_SINGULAR_PI;
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int r = c + 1; r < d; ++r)
            if (std::fabs(A[r * d + c]) > std::fabs(A[piv * d + c])) piv = r;
        if (std::fabs(A[piv * d + c]) <= 1e-12 * scale) return IWFPM_ERR_SINGULAR_PI;
        if (piv != c) {
            for (int j = 0; j < d; ++j) std::swap(A[c * d + j], A[piv * d + j]);
            for (int j = 0; j < m; ++j) std::swap(B[c * m + j], B[piv * m + j]);
        }
        for (int r = c + 1; r < d; ++r) {
            double f = A[r * d + c] / A[c * d + c];
            if (f == 0.0) continue;
            for (int j = c; j < d; ++j) A[r * d + j] -= f * A[c * d + j];
            for (int j = 0; j < m; ++j) B[r * m + j] -= f * B[c * m + j];
        }
    }
    Q.assign(d * m, 0.0);
    for (int j = 0; j < m; ++j) {
        for (int r = d - 1; r >= 0; --r) {
            double s = B[r * m + j];
            for (int c = r + 1; c < d; ++c) s -= A[r * d + c] * Q[c * m + j];
            Q[r * m + j] = s / A[r * d + r];
        }
    }
    // P_I Q = P_II should hold; a rank-deficient P_I would have stopped above.
    return IWFPM_OK;
}

// storage axis of paper index j (0-based): k_I axes are the last d
static int axis_of(int d, int n, int j) { return j < d ? (n - d) + j : j - d; }

void host_label(const iwfpm_plan_s* p, long long gpos, int* k) {
    const DevGeom& g = p->geom;
    const int d = p->d, n = p->n;
    long long s = gpos / g.nkI;
    long long r = gpos - s * g.nkI;
    // k_II from the slice index (eq:inverse2)
    long long t = s;
    for (int ax = n - d - 1; ax >= 0; --ax) {
        int E = g.ext[ax];
        int ks = (int)(t % E);
        t /= E;
        int Lj = E / 2;
        k[d + ax] = ks < Lj ? ks : ks - E;
    }
    for (int j = d - 1; j >= 0; --j) {
        int ax = n - d + j;
        int E = g.ext[ax];
        int ks = (int)(r % E);
        r /= E;
        int a = p->slice_a[s * d + j];
        int m = (ks - a) % E;
        if (m < 0) m += E;
        k[j] = a + m;
    }
}

long long host_grid_to_vec(const iwfpm_plan_s* p, long long gpos) {
    if (p->opts.order == IWFPM_ORDER_GRID) return gpos;
    const DevGeom& g = p->geom;
    const int d = p->d, n = p->n;
    long long s = gpos / g.nkI;
    long long r = gpos - s * g.nkI;
    long long out = s * g.nkI;
    for (int j = d - 1; j >= 0; --j) {
        int ax = n - d + j;
        int E = g.ext[ax];
        int ks = (int)(r % E);
        r /= E;
        int m = (ks - p->slice_a[s * d + j]) % E;
        if (m < 0) m += E;
        out += (long long)m * g.stride[ax];
    }
    return out;
}

double host_kinetic(const iwfpm_plan_s* p, const int* k) {
    double tot = 0.0;
    for (int j = 0; j < p->d; ++j) {
        double acc = 0.0;
        for (int i = 0; i < p->n; ++i) acc += p->P[j * p->n + i] * (double)k[i];
        double v = kTwoPi * acc;
        tot += v * v;
    }
    return 0.5 * tot;
}

static int build_geometry(iwfpm_plan_s* p) {
    const int d = p->d, n = p->n;
    DevGeom& g = p->geom;
    std::memset(&g, 0, sizeof(g));
    g.n = n;
    g.d = d;
    g.order = p->opts.order;
    g.kin = 1;
    for (int ax = 0; ax < n; ++ax) {
        int e = ax < n - d ? 2 * p->L[ax] : 2 * p->K[ax - (n - d)];
        g.ext[ax] = e;
    }
    long long st = 1;
    for (int ax = n - 1; ax >= 0; --ax) {
        g.stride[ax] = st;
        st *= g.ext[ax];
        if (st > (1LL << 31) - 1) return IWFPM_ERR_UNSUPPORTED;
    }
    g.N = st;
    // stages of the long axes and their twiddle tables e^{+2 pi i j / ext}
    p->tw.clear();
    for (int ax = 0; ax < n; ++ax) {
        g.nfac[ax] = axis_factors(g.ext[ax], g.fac[ax]);
        if (g.nfac[ax] == 0) return IWFPM_ERR_UNSUPPORTED;
        g.twoff[ax] = 0;
        if (g.nfac[ax] > 1) {
            g.twoff[ax] = (int)(p->tw.size() / 2);
            const int E = g.ext[ax];
            for (int j = 0; j < E; ++j) {
                // in long double, then rounded once
                const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)E;
                p->tw.push_back((double)std::cos(a));
                p->tw.push_back((double)std::sin(a));
            }
        }
    }
    g.nkI = 1;
    for (int ax = n - d; ax < n; ++ax) g.nkI *= g.ext[ax];
    for (int j = 0; j < d; ++j)
        for (int i = 0; i < d; ++i) g.P1[j * d + i] = kTwoPi * p->P[j * n + i];

    // per-slice tables: q = Q k_II, the window's lower end a = -K - floor(q)
    // (the floor form of eq:inverse3), and 2 pi P_II k_II for the kinetic term
    p->nslice = g.N / g.nkI;
    p->slice_a.assign(p->nslice * d, 0);
    p->slice_g.assign(p->nslice * d, 0.0);
    const int m = n - d;
    std::vector<int> kII(m);
    for (long long s = 0; s < p->nslice; ++s) {
        long long t = s;
        for (int ax = m - 1; ax >= 0; --ax) {
            int E = g.ext[ax];
            int ks = (int)(t % E);
            t /= E;
            kII[ax] = ks < E / 2 ? ks : ks - E;
        }
        for (int j = 0; j < d; ++j) {
            double q = 0.0;
            for (int i = 0; i < m; ++i) q = q + p->Q[j * m + i] * (double)kII[i];
            // snap values within rounding of an integer onto it, so that the
            // half-open window rule decides exact ties the same way every time
            double rq = std::nearbyint(q);
            if (std::fabs(q - rq) <= 1e-12 * std::max(1.0, std::fabs(q))) q = rq;
            double qe = q;
            if (p->opts.window_variant == IWFPM_WINDOW_ROUNDED) qe = std::floor(q + 0.5);
            if (p->opts.window_variant == IWFPM_WINDOW_PM) qe = 0.0;
            p->slice_a[s * d + j] = -p->K[j] - (int)std::floor(qe);
            double acc = 0.0;
            for (int i = 0; i < m; ++i) acc = acc + p->P[j * n + d + i] * (double)kII[i];
            p->slice_g[s * d + j] = kTwoPi * acc;
        }
    }
    return IWFPM_OK;
}

static int build_potential(iwfpm_plan_s* p, int n_modes, const int32_t* modes, const double* vhat) {
    const int n = p->n, d = p->d;
    // merge duplicate modes
    std::map<std::vector<int>, std::pair<double, double>> acc;
    for (int i = 0; i < n_modes; ++i) {
        std::vector<int> m(modes + (size_t)i * n, modes + (size_t)(i + 1) * n);
        auto& v = acc[m];
        v.first += vhat[2 * i];
        v.second += vhat[2 * i + 1];
    }
    p->modes.clear();
    p->vre.clear();
    p->vim.clear();
    p->vhat0 = 0.0;
    p->vsum_nonzero = 0.0;
    p->vsum_abs = 0.0;
    for (auto& kv : acc) {
        const std::vector<int>& m = kv.first;
        std::vector<int> mm(n);
        for (int j = 0; j < n; ++j) mm[j] = -m[j];
        auto it = acc.find(mm);
        double re = kv.second.first, im = kv.second.second;
        double tol = 1e-12 * std::max(1.0, std::hypot(re, im));
        if (it == acc.end() || std::fabs(it->second.first - re) > tol || std::fabs(it->second.second + im) > tol)
            return IWFPM_ERR_NONHERMITIAN;
        bool zero = true;
        for (int j = 0; j < n; ++j) zero = zero && m[j] == 0;
        double a = std::hypot(re, im);
        if (zero) p->vhat0 = re;
        else p->vsum_nonzero += a;
        p->vsum_abs += a;
        p->modes.insert(p->modes.end(), m.begin(), m.end());
        p->vre.push_back(re);
        p->vim.push_back(im);
    }
    const int nm = (int)p->vre.size();
    const DevGeom& g = p->geom;
    bool axis_aligned = true;
    for (int i = 0; i < nm && axis_aligned; ++i) {
        int nz = 0;
        for (int j = 0; j < n; ++j) nz += p->modes[i * n + j] != 0;
        axis_aligned = nz <= 1;
    }
    const double invN = 1.0 / (double)g.N;
    if (axis_aligned) {
        // V(y_l) = sum over axes of f_ax(l_ax), f built from that axis' modes
        p->geom.vmode = 0;
        int off = 0;
        for (int ax = 0; ax < n; ++ax) {
            p->geom.voff[ax] = off;
            off += g.ext[ax];
        }
        std::vector<double> tre(off, 0.0), tim(off, 0.0);
        for (int i = 0; i < nm; ++i) {
            int jnz = -1;
            for (int j = 0; j < n; ++j)
                if (p->modes[i * n + j] != 0) jnz = j;
            int ax = jnz < 0 ? 0 : axis_of(d, n, jnz);
            int t = jnz < 0 ? 0 : p->modes[i * n + jnz];
            int E = g.ext[ax];
            for (int l = 0; l < E; ++l) {
                long long ph = ((long long)t * l) % E;
                if (ph < 0) ph += E;
                double ang = kTwoPi * (double)ph / (double)E;
                double c = std::cos(ang), s = std::sin(ang);
                tre[p->geom.voff[ax] + l] += p->vre[i] * c - p->vim[i] * s;
                tim[p->geom.voff[ax] + l] += p->vre[i] * s + p->vim[i] * c;
            }
        }
        p->vtab.resize(off);
        for (int i = 0; i < off; ++i) p->vtab[i] = tre[i] * invN;
        p->vgrid.clear();
    } else {
        p->geom.vmode = 1;
        p->vgrid.assign(g.N, 0.0);
        std::vector<int> l(n);
        for (long long gp = 0; gp < g.N; ++gp) {
            long long t = gp;
            for (int ax = n - 1; ax >= 0; --ax) {
                l[ax] = (int)(t % g.ext[ax]);
                t /= g.ext[ax];
            }
            double v = 0.0;
            for (int i = 0; i < nm; ++i) {
                double ph = 0.0;
                for (int j = 0; j < n; ++j) {
                    int ax = axis_of(d, n, j);
                    long long pj = ((long long)p->modes[i * n + j] * l[ax]) % g.ext[ax];
                    if (pj < 0) pj += g.ext[ax];
                    ph += (double)pj / (double)g.ext[ax];
                }
                double ang = kTwoPi * (ph - std::floor(ph));
                v += p->vre[i] * std::cos(ang) - p->vim[i] * std::sin(ang);
            }
            p->vgrid[gp] = v * invN;
        }
        p->vtab.clear();
    }
    return IWFPM_OK;
}

static const size_t kLdsDefault = 64 * 1024;
static const size_t kLdsMax = 160 * 1024;

static int round64(int x) { return ((x + 63) / 64) * 64; }
static void finalize_threepass(const iwfpm_plan_s* p, Schedule& sc, int prec, int outer_threads = 0);
static int choose_mid_schedule(iwfpm_plan_s* p, int prec);

static int choose_schedule(iwfpm_plan_s* p, int prec) {
    Schedule& sc = p->sched[prec];
    const DevGeom& g = p->geom;
    const int n = p->n;
    const size_t esz = prec == 1 ? 8 : 16;
    int maxcls = 16;
    for (int ax = 0; ax < n; ++ax) maxcls = std::max(maxcls, axis_class(g, ax));
    sc.maxs_fused = maxcls;
    const size_t lf = lds_fused(g, esz);
    bool want_fused = p->opts.schedule == IWFPM_SCHED_FUSED ||
                      (p->opts.schedule == IWFPM_SCHED_AUTO && lf <= kLdsDefault);
    if (want_fused) {
        if (lf > kLdsMax) return IWFPM_ERR_UNSUPPORTED;
        sc.fused = true;
        int maxp = 0;
        for (int ax = 0; ax < n; ++ax) maxp = std::max(maxp, axis_items(g, ax, g.N));
        sc.threads_fused = std::min(256, round64(maxp));
        return IWFPM_OK;
    }
    sc.fused = false;
    if (n < 2) return IWFPM_ERR_UNSUPPORTED;
    // pick the split: trailing axes [split, n) form the contiguous slabs
    int lo = 1, hi = n - 1;
    if (p->opts.order == IWFPM_ORDER_WINDOW) hi = n - p->d;  // k_I axes must stay in one slab
    PassDesc& pd = sc.pd;
    pd.xcd_remap = 1;
    int split = 0;
    if (p->opts.split > 0) {
        split = p->opts.split;
        if (split < lo || split > hi) return IWFPM_ERR_ARG;
    } else {
        // prefer the k_I / k_II boundary, then the most balanced feasible split
        double best = 1e300;
        for (int s = lo; s <= hi; ++s) {
            PassDesc t{};
            t.s_in = g.stride[s - 1];
            t.s_out = g.N / t.s_in;
            t.slabs_per_wg = 1;
            t.tile = 1;
            t.split = s;
            if (lds_slabs(g, t, esz) > kLdsMax || lds_columns(g, t, esz) > kLdsMax) continue;
            double cost = std::fabs(std::log((double)t.s_in) - std::log((double)t.s_out));
            if (s == n - p->d) cost -= 0.5;
            if (cost < best) {
                best = cost;
                split = s;
            }
        }
        if (split == 0) return choose_mid_schedule(p, prec);
    }
    pd.split = split;
    pd.split_mid = 0;
    pd.s_in = g.stride[split - 1];
    pd.s_out = g.N / pd.s_in;
    // middle pass: `tile` consecutive columns (a power of two)
    int T = p->opts.tile;
    if (T > 0 && (T & (T - 1))) return IWFPM_ERR_ARG;
    if (T > 0) {
        pd.tile = T;
        if (lds_columns(g, pd, esz) > kLdsMax) T = 0;  // does not fit this precision: choose here
    }
    if (T <= 0) {
        // widest tile (<= 16 columns) of which two workgroups still fit one CU's LDS
        T = 1;
        for (;;) {
            pd.tile = 2 * T;
            if (2 * T > 16 || lds_columns(g, pd, esz) > kLdsMax / 2 || 2 * T > pd.s_in) break;
            T *= 2;
        }
    }
    pd.tile = T;
    if (lds_columns(g, pd, esz) > kLdsMax) return IWFPM_ERR_UNSUPPORTED;
    // slabs per workgroup for passes 1 and 3: up to ~40 KB of LDS each, and
    // enough pencils per axis to keep a few waves busy
    int G = 1;
    for (;;) {
        pd.slabs_per_wg = 2 * G;
        if (2 * G > 64 || 2 * G > pd.s_out || lds_slabs(g, pd, esz) > kLdsDefault * 5 / 8) break;
        G *= 2;
    }
    pd.slabs_per_wg = G;
    if (lds_slabs(g, pd, esz) > kLdsMax) return IWFPM_ERR_UNSUPPORTED;
    finalize_threepass(p, sc, prec);
    return IWFPM_OK;
}

// threads and extent classes of a three-pass schedule whose split, tile and
// slabs per workgroup are set; the middle pass gets outer_threads threads
// (0: as many as it has pencils, up to its class's largest workgroup)
static void finalize_threepass(const iwfpm_plan_s* p, Schedule& sc, int prec, int outer_threads) {
    const DevGeom& g = p->geom;
    PassDesc& pd = sc.pd;
    int maxpi = 0, maxpo = 0, mi = 16, mo = 16;
    for (int ax = pd.split; ax < p->n; ++ax) {
        maxpi = std::max(maxpi, axis_items(g, ax, (long long)pd.slabs_per_wg * pd.s_in));
        mi = std::max(mi, axis_class(g, ax));
    }
    for (int ax = 0; ax < pd.split; ++ax) {
        maxpo = std::max(maxpo, axis_items(g, ax, (long long)pd.s_out * pd.tile));
        mo = std::max(mo, axis_class(g, ax));
    }
    pd.threads_inner = std::min(256, round64(maxpi));
    const int cap = wide_pass_threads(prec, mo);
    pd.threads_outer = std::min(outer_threads > 0 ? std::min(outer_threads, cap) : cap, round64(maxpo));
    sc.maxs_inner = mi;
    sc.maxs_outer = mo;
    sc.fused = false;
    sc.ok = true;
}

// threads and extent classes of a schedule with the further pass
static void finalize_mid(const iwfpm_plan_s* p, Schedule& sc, int prec) {
    const DevGeom& g = p->geom;
    PassDesc& pd = sc.pd;
    const PassDesc q = middle_desc(g, pd);
    const int mid = g.stride[pd.split_mid - 1] / pd.s_in;
    int maxpi = 0, maxpo = 0, maxpm = 0, mi = 16, mo = 16;
    for (int ax = pd.split; ax < p->n; ++ax) {
        maxpi = std::max(maxpi, axis_items(g, ax, (long long)pd.slabs_per_wg * pd.s_in));
        mi = std::max(mi, axis_class(g, ax));
    }
    for (int ax = 0; ax < pd.split_mid; ++ax) {
        maxpo = std::max(maxpo, axis_items(g, ax, (long long)q.s_out * pd.tile));
        mo = std::max(mo, axis_class(g, ax));
    }
    for (int ax = pd.split_mid; ax < pd.split; ++ax) {
        maxpm = std::max(maxpm, axis_items(g, ax, (long long)mid * pd.tile_mid));
        mo = std::max(mo, axis_class(g, ax));
    }
    pd.threads_inner = std::min(256, round64(maxpi));
    pd.threads_outer = std::min(wide_pass_threads(prec, mo), round64(maxpo));
    pd.threads_mid = std::min(wide_pass_threads(prec, mo), round64(maxpm));
    sc.maxs_inner = mi;
    sc.maxs_outer = mo;
    sc.fused = false;
    sc.ok = true;
}

// Grids whose leading block fits no single middle pass (e.g. 40^3 x 10^3):
// passes 1 and 3 keep the trailing axes [split, n), the middle pass the
// leading axes [0, s1) with the potential, and a further pass the axes
// [s1, split) in between (five launches per apply instead of three).
static int choose_mid_schedule(iwfpm_plan_s* p, int prec) {
    Schedule& sc = p->sched[prec];
    const DevGeom& g = p->geom;
    const int n = p->n;
    const size_t esz = prec == 1 ? 8 : 16;
    const int hi = p->opts.order == IWFPM_ORDER_WINDOW ? n - p->d : n - 1;
    PassDesc& pd = sc.pd;
    pd = PassDesc{};
    pd.xcd_remap = 1;
    // the largest slab that fits (the most axes in passes 1 and 3, which move
    // whole contiguous slabs), then the most balanced cut of the leading block
    for (int split = 2; split <= hi; ++split) {
        PassDesc t{};
        t.split = split;
        t.s_in = g.stride[split - 1];
        t.s_out = g.N / t.s_in;
        t.slabs_per_wg = 1;
        t.tile = 1;
        t.tile_mid = 1;
        if (lds_slabs(g, t, esz) > kLdsMax) continue;
        int best_s1 = 0;
        double best = 1e300;
        for (int s1 = 1; s1 < split; ++s1) {
            t.split_mid = s1;
            if (lds_columns(g, middle_desc(g, t), esz) > kLdsMax || lds_mid(g, t, esz) > kLdsMax) continue;
            const double outer = (double)(g.N / g.stride[s1 - 1]);
            const double mid = (double)(g.stride[s1 - 1] / t.s_in);
            const double cost = std::fabs(std::log(outer) - std::log(mid));
            if (cost < best) {
                best = cost;
                best_s1 = s1;
            }
        }
        if (best_s1 == 0) continue;
        pd.split = split;
        pd.s_in = t.s_in;
        pd.s_out = t.s_out;
        pd.split_mid = best_s1;
        break;
    }
    if (pd.split == 0) return IWFPM_ERR_UNSUPPORTED;
    // widest tiles (<= 64 columns) of which two workgroups fit one CU's LDS:
    // a short block (one 40-point axis) needs many columns to give every lane
    // of a wave a pencil
    const PassDesc q0 = middle_desc(g, pd);
    int T = 1;
    for (;;) {
        pd.tile = 2 * T;
        if (2 * T > 64 || 2 * T > q0.s_in || lds_columns(g, middle_desc(g, pd), esz) > kLdsMax / 2) break;
        T *= 2;
    }
    pd.tile = T;
    int Tm = 1;
    for (;;) {
        pd.tile_mid = 2 * Tm;
        if (2 * Tm > 64 || 2 * Tm > pd.s_in || lds_mid(g, pd, esz) > kLdsMax / 2) break;
        Tm *= 2;
    }
    pd.tile_mid = Tm;
    int G = 1;
    for (;;) {
        pd.slabs_per_wg = 2 * G;
        if (2 * G > 64 || 2 * G > pd.s_out || lds_slabs(g, pd, esz) > kLdsDefault * 5 / 8) break;
        G *= 2;
    }
    pd.slabs_per_wg = G;
    if (lds_columns(g, middle_desc(g, pd), esz) > kLdsMax || lds_mid(g, pd, esz) > kLdsMax ||
        lds_slabs(g, pd, esz) > kLdsMax)
        return IWFPM_ERR_UNSUPPORTED;
    finalize_mid(p, sc, prec);
    return IWFPM_OK;
}

// every feasible schedule for precision prec
static std::vector<Schedule> schedule_candidates(const iwfpm_plan_s* p, int prec) {
    std::vector<Schedule> out;
    const DevGeom& g = p->geom;
    const int n = p->n;
    const size_t esz = prec == 1 ? 8 : 16;
    if (lds_fused(g, esz) <= kLdsMax) {
        Schedule f = p->sched[prec];
        int maxcls = 16, maxp = 0;
        for (int ax = 0; ax < n; ++ax) {
            maxcls = std::max(maxcls, axis_class(g, ax));
            maxp = std::max(maxp, axis_items(g, ax, g.N));
        }
        f.fused = true;
        f.ok = true;
        f.maxs_fused = maxcls;
        f.threads_fused = std::min(256, round64(maxp));
        out.push_back(f);
    }
    if (n < 2) return out;
    int hi = p->opts.order == IWFPM_ORDER_WINDOW ? n - p->d : n - 1;
    for (int split = 1; split <= hi; ++split) {
        for (int T = 1; T <= 32; T *= 2) {
            for (int G = 1; G <= 64; G *= 2) {
                Schedule c{};
                PassDesc& pd = c.pd;
                pd.split = split;
                pd.s_in = g.stride[split - 1];
                pd.s_out = g.N / pd.s_in;
                pd.tile = T;
                pd.slabs_per_wg = G;
                pd.xcd_remap = 1;
                if (T > pd.s_in || G > pd.s_out) continue;
                if (lds_columns(g, pd, esz) > kLdsMax || lds_slabs(g, pd, esz) > kLdsMax) continue;
                // middle-pass workgroups of 256, 512 and 1024 threads (as far
                // as the class and the pencils allow; duplicates dropped)
                int last = 0;
                for (int th = 256; th <= 1024; th *= 2) {
                    Schedule t = c;
                    finalize_threepass(p, t, prec, th);
                    if (t.pd.threads_outer == last) continue;
                    last = t.pd.threads_outer;
                    out.push_back(t);
                }
            }
        }
    }
    // no three-pass schedule fits: the plan's own schedule with the further pass
    if (out.empty() && p->sched[prec].ok && p->sched[prec].pd.split_mid > 0) out.push_back(p->sched[prec]);
    return out;
}

template <typename R>
static int prepare_kernels() {
    int b = (int)kLdsMax;
    hipError_t e = hipSuccess;
    e = prepare_fused<R, 16>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_fused<R, 32>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_fused<R, 64>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_pass1<R, 16>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_pass1<R, 32>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_pass1<R, 64>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_pass2<R, 16>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_pass2<R, 32>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_pass2<R, 64>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_pass3<R, 16>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_pass3<R, 32>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_pass3<R, 64>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_passm<R, 16>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_passm<R, 32>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_passm<R, 64>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_batch<R, 16>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_batch<R, 32>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    e = prepare_batch<R, 64>(b); if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    return IWFPM_OK;
}

template <typename T>
static int upload(DeviceBuf& b, const std::vector<T>& v) {
    if (v.empty()) return IWFPM_OK;
    int rc = dev_alloc(b, v.size() * sizeof(T));
    if (rc != IWFPM_OK) return rc;
    if (hipMemcpy(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    return IWFPM_OK;
}

static int upload_tables(iwfpm_plan_s* p) {
    int rc;
    if ((rc = upload(p->d_slice_a, p->slice_a)) != IWFPM_OK) return rc;
    if ((rc = upload(p->d_slice_g, p->slice_g)) != IWFPM_OK) return rc;
    std::vector<float> f32;
    if (!p->vtab.empty()) {
        if ((rc = upload(p->d_vtab64, p->vtab)) != IWFPM_OK) return rc;
        f32.assign(p->vtab.begin(), p->vtab.end());
        if ((rc = upload(p->d_vtab32, f32)) != IWFPM_OK) return rc;
    }
    if (!p->vgrid.empty()) {
        if ((rc = upload(p->d_vgrid64, p->vgrid)) != IWFPM_OK) return rc;
        f32.assign(p->vgrid.begin(), p->vgrid.end());
        if ((rc = upload(p->d_vgrid32, f32)) != IWFPM_OK) return rc;
    }
    if (!p->tw.empty()) {
        if ((rc = upload(p->d_tw64, p->tw)) != IWFPM_OK) return rc;
        f32.assign(p->tw.begin(), p->tw.end());
        if ((rc = upload(p->d_tw32, f32)) != IWFPM_OK) return rc;
    }
    p->tabs.tw32 = (const float*)p->d_tw32.ptr;
    p->tabs.tw64 = (const double*)p->d_tw64.ptr;
    p->tabs.slice_a = (const int*)p->d_slice_a.ptr;
    p->tabs.slice_g = (const double*)p->d_slice_g.ptr;
    p->tabs.vtab32 = (const float*)p->d_vtab32.ptr;
    p->tabs.vtab64 = (const double*)p->d_vtab64.ptr;
    p->tabs.vgrid32 = (const float*)p->d_vgrid32.ptr;
    p->tabs.vgrid64 = (const double*)p->d_vgrid64.ptr;
    return IWFPM_OK;
}

static void prof_collect(ApplyProfiler::Slot& s, ApplyProfiler& pr) {
    if (!s.pending) return;
    (void)hipEventSynchronize(s.ev[s.kind ? 3 : 1]);
    float t = 0.f;
    if (s.kind == 0) {
        if (hipEventElapsedTime(&t, s.ev[0], s.ev[1]) == hipSuccess) pr.ms[0] += t;
        pr.launches[0] += 1;
        pr.points[0] += s.points;
    } else {
        for (int k = 0; k < 3; ++k) {
            if (hipEventElapsedTime(&t, s.ev[k], s.ev[k + 1]) == hipSuccess) pr.ms[k + 1] += t;
            pr.launches[k + 1] += 1;
            pr.points[k + 1] += s.points;
        }
    }
    s.pending = false;
}

// event to record after kernel `i` of this launch sequence (or null)
static hipEvent_t* prof_slot(ApplyProfiler* pr, bool fused, long long points, hipStream_t st) {
    if (!pr || !pr->on) return nullptr;
    if (pr->ring.empty()) return nullptr;
    ApplyProfiler::Slot& s = pr->ring[pr->head];
    pr->head = (pr->head + 1) % pr->ring.size();
    prof_collect(s, *pr);
    s.kind = fused ? 0 : 1;
    s.points = points;
    s.pending = true;
    (void)hipEventRecord(s.ev[0], st);
    return s.ev;
}

template <typename R>
static hipError_t launch_sched(const Schedule& sc, const DevGeom& g, const DevTabs& t, const void* psi, void* hpsi,
                               void* ws, int nvec, hipStream_t st, ApplyProfiler* pr) {
    hipEvent_t* ev = prof_slot(pr, sc.fused, (long long)nvec * g.N, st);
    if (sc.fused) {
        hipError_t e;
        switch (sc.maxs_fused) {
            case 16: e = launch_fused<R, 16>(g, t, sc.threads_fused, psi, hpsi, nvec, st); break;
            case 32: e = launch_fused<R, 32>(g, t, sc.threads_fused, psi, hpsi, nvec, st); break;
            default: e = launch_fused<R, 64>(g, t, sc.threads_fused, psi, hpsi, nvec, st); break;
        }
        if (ev) (void)hipEventRecord(ev[1], st);
        return e;
    }
    hipError_t e;
    switch (sc.maxs_inner) {
        case 16: e = launch_pass1<R, 16>(g, t, sc.pd, psi, ws, nvec, st); break;
        case 32: e = launch_pass1<R, 32>(g, t, sc.pd, psi, ws, nvec, st); break;
        default: e = launch_pass1<R, 64>(g, t, sc.pd, psi, ws, nvec, st); break;
    }
    if (ev) (void)hipEventRecord(ev[1], st);
    if (e != hipSuccess) return e;
    // with the further pass: its inverse half, the middle pass on the leading
    // axes, its forward half (timed together as the middle stage)
    const bool mid = sc.pd.split_mid > 0;
    auto passm = [&](int sign) {
        switch (sc.maxs_outer) {
            case 16: return launch_passm<R, 16>(g, t, sc.pd, sign, ws, nvec, st);
            case 32: return launch_passm<R, 32>(g, t, sc.pd, sign, ws, nvec, st);
            default: return launch_passm<R, 64>(g, t, sc.pd, sign, ws, nvec, st);
        }
    };
    if (mid && (e = passm(+1)) != hipSuccess) return e;
    const PassDesc q = middle_desc(g, sc.pd);
    switch (sc.maxs_outer) {
        case 16: e = launch_pass2<R, 16>(g, t, q, ws, nvec, st); break;
        case 32: e = launch_pass2<R, 32>(g, t, q, ws, nvec, st); break;
        default: e = launch_pass2<R, 64>(g, t, q, ws, nvec, st); break;
    }
    if (e != hipSuccess) return e;
    if (mid && (e = passm(-1)) != hipSuccess) return e;
    if (ev) (void)hipEventRecord(ev[2], st);
    switch (sc.maxs_inner) {
        case 16: e = launch_pass3<R, 16>(g, t, sc.pd, psi, ws, hpsi, nvec, st); break;
        case 32: e = launch_pass3<R, 32>(g, t, sc.pd, psi, ws, hpsi, nvec, st); break;
        default: e = launch_pass3<R, 64>(g, t, sc.pd, psi, ws, hpsi, nvec, st); break;
    }
    if (ev) (void)hipEventRecord(ev[3], st);
    return e;
}

static const size_t kWorkspaceCap = (size_t)4 << 30;

int plan_ensure_ws(iwfpm_plan_s* p, int nvec, int prec, hipStream_t st) {
    const Schedule& sc = p->sched[prec];
    if (!sc.ok) return IWFPM_ERR_UNSUPPORTED;
    if (sc.fused) return IWFPM_OK;
    size_t need = (size_t)p->geom.N * (prec ? 8 : 16) * nvec;
    if (p->d_ws.bytes < need) {
        if (hipStreamSynchronize(st) != hipSuccess) return IWFPM_ERR_DEVICE;
        if (dev_alloc(p->d_ws, need) != IWFPM_OK) return IWFPM_ERR_ALLOC;
    }
    return IWFPM_OK;
}

int plan_apply_ws(iwfpm_plan_s* p, const void* psi, void* hpsi, int nvec, int precision, hipStream_t st,
                  int kinetic, void* ws, size_t ws_bytes) {
    if (nvec == 0) return IWFPM_OK;
    const int prec = precision == IWFPM_PREC_FP32 ? 1 : 0;
    const Schedule& sc = p->sched[prec];
    if (!sc.ok) return IWFPM_ERR_UNSUPPORTED;
    const size_t esz = prec ? 8 : 16;
    const long long N = p->geom.N;
    int chunk = nvec;
    if (!sc.fused) {
        const size_t per = (size_t)N * esz;
        if (per > ws_bytes || !ws) return IWFPM_ERR_ARG;
        chunk = (int)std::min<size_t>((size_t)nvec, ws_bytes / per);
    }
    const double2* x = reinterpret_cast<const double2*>(psi);
    double2* y = reinterpret_cast<double2*>(hpsi);
    for (int v0 = 0; v0 < nvec; v0 += chunk) {
        int nv = std::min(chunk, nvec - v0);
        DevGeom g = p->geom;
        g.kin = kinetic ? 1 : 0;
        hipError_t e = prec ? launch_sched<float>(sc, g, p->tabs, x + (size_t)v0 * N, y + (size_t)v0 * N,
                                                  ws, nv, st, kinetic ? &p->prof : nullptr)
                            : launch_sched<double>(sc, g, p->tabs, x + (size_t)v0 * N, y + (size_t)v0 * N,
                                                   ws, nv, st, kinetic ? &p->prof : nullptr);
        if (e != hipSuccess) return IWFPM_ERR_DEVICE;
    }
    return IWFPM_OK;
}

int plan_apply(iwfpm_plan_s* p, const void* psi, void* hpsi, int nvec, int precision, hipStream_t st, int kinetic) {
    if (nvec == 0) return IWFPM_OK;
    const int prec = precision == IWFPM_PREC_FP32 ? 1 : 0;
    const Schedule& sc = p->sched[prec];
    if (!sc.ok) return IWFPM_ERR_UNSUPPORTED;
    if (!sc.fused) {
        // the plan's own workspace, grown to the vectors of one chunk
        const size_t per = (size_t)p->geom.N * (prec ? 8 : 16);
        const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)nvec, kWorkspaceCap / per));
        const size_t need = per * chunk;
        if (p->d_ws.bytes < need) {
            if (hipStreamSynchronize(st) != hipSuccess) return IWFPM_ERR_DEVICE;
            if (dev_alloc(p->d_ws, need) != IWFPM_OK) return IWFPM_ERR_ALLOC;
        }
        return plan_apply_ws(p, psi, hpsi, nvec, precision, st, kinetic, p->d_ws.ptr, need);
    }
    return plan_apply_ws(p, psi, hpsi, nvec, precision, st, kinetic, nullptr, 0);
}

}  // namespace iwfpm

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void iwfpm_default_opts(iwfpm_opts* o) {
    if (!o) return;
    o->precision = IWFPM_PREC_FP64;
    o->window_variant = IWFPM_WINDOW_EXACT;
    o->order = IWFPM_ORDER_GRID;
    o->device = 0;
    o->schedule = IWFPM_SCHED_AUTO;
    o->split = 0;
    o->tile = 0;
}

const char* iwfpm_status_string(int s) {
    switch (s) {
        case IWFPM_OK: return "ok";
        case IWFPM_ERR_ARG: return "invalid argument";
        case IWFPM_ERR_SINGULAR_PI: return "P_I is singular";
        case IWFPM_ERR_NONHERMITIAN: return "potential modes do not describe a real potential";
        case IWFPM_ERR_UNSUPPORTED: return "unsupported by this library";
        case IWFPM_ERR_ALLOC: return "allocation failed";
        case IWFPM_ERR_DEVICE: return "HIP error";
        case IWFPM_ERR_NUMERIC: return "numerical breakdown";
        case IWFPM_ERR_NOCONV: return "not converged";
        case IWFPM_ERR_WEIGHTS: return "learned preconditioner weights missing or invalid";
        case IWFPM_ERR_NODEVICE: return "host-only plan";
        case IWFPM_ERR_TOO_LARGE: return "one vector's intermediate grid exceeds the static scratch array";
        default: return "unknown status";
    }
}

int iwfpm_plan(int d, int n, const double* P, const int32_t* K, const int32_t* L, int n_modes,
               const int32_t* modes, const double* vhat, const iwfpm_opts* opts, iwfpm_plan_t* out) {
    if (!out) return IWFPM_ERR_ARG;
    *out = nullptr;
    if (d < 1 || n <= d || n > kMaxAxes || !P || !K || !L || n_modes < 0) return IWFPM_ERR_ARG;
    if (n_modes > 0 && (!modes || !vhat)) return IWFPM_ERR_ARG;
    iwfpm_opts o;
    iwfpm_default_opts(&o);
    if (opts) o = *opts;
    if (o.precision < 0 || o.precision > 1 || o.window_variant < 0 || o.window_variant > 2 || o.order < 0 ||
        o.order > 1 || o.schedule < 0 || o.schedule > 2 || o.device < -1)
        return IWFPM_ERR_ARG;
    for (int i = 0; i < d * n; ++i)
        if (!std::isfinite(P[i])) return IWFPM_ERR_ARG;
    for (int j = 0; j < d; ++j)
        if (K[j] < 1 || !extent_supported(2 * K[j])) return K[j] < 1 ? IWFPM_ERR_ARG : IWFPM_ERR_UNSUPPORTED;
    for (int j = 0; j < n - d; ++j)
        if (L[j] < 1 || !extent_supported(2 * L[j])) return L[j] < 1 ? IWFPM_ERR_ARG : IWFPM_ERR_UNSUPPORTED;
    for (int i = 0; i < 2 * n_modes; ++i)
        if (!std::isfinite(vhat[i])) return IWFPM_ERR_ARG;

    iwfpm_plan_s* p = new (std::nothrow) iwfpm_plan_s();
    if (!p) return IWFPM_ERR_ALLOC;
    p->d = d;
    p->n = n;
    p->opts = o;
    p->P.assign(P, P + d * n);
    p->K.assign(K, K + d);
    p->L.assign(L, L + (n - d));
    int rc = solve_Q(d, n, P, p->Q);
    if (rc == IWFPM_OK) rc = build_geometry(p);
    if (rc == IWFPM_OK) rc = build_potential(p, n_modes, modes, vhat);
    if (rc == IWFPM_OK) {
        // a precision whose tiles do not fit is reported at apply time only
        int r64 = choose_schedule(p, 0), r32 = choose_schedule(p, 1);
        p->sched[0].ok = r64 == IWFPM_OK;
        p->sched[1].ok = r32 == IWFPM_OK;
        if (r64 == IWFPM_ERR_ARG || r32 == IWFPM_ERR_ARG) rc = IWFPM_ERR_ARG;
        else if (!p->sched[o.precision].ok) rc = o.precision ? r32 : r64;
    }
    if (rc != IWFPM_OK) {
        delete p;
        return rc;
    }
    // max Lambda over the grid for the norm bound
    {
        std::vector<int> k(n);
        double mx = 0.0;
        for (long long gp = 0; gp < p->geom.N; ++gp) {
            host_label(p, gp, k.data());
            mx = std::max(mx, host_kinetic(p, k.data()));
        }
        p->lam_max = mx;
    }
    if (o.device >= 0) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || o.device >= ndev) {
            (void)hipGetLastError();
            delete p;
            return IWFPM_ERR_DEVICE;
        }
        DeviceGuard guard(o.device);
        if (!guard.ok) {
            delete p;
            return IWFPM_ERR_DEVICE;
        }
        rc = prepare_kernels<float>();
        if (rc == IWFPM_OK) rc = prepare_kernels<double>();
        if (rc == IWFPM_OK) rc = upload_tables(p);
        if (rc != IWFPM_OK) {
            iwfpm_destroy(p);
            return rc;
        }
        p->host_only = false;
    }
    *out = p;
    return IWFPM_OK;
}

int iwfpm_dof(iwfpm_plan_t p, int64_t* N) {
    if (!p || !N) return IWFPM_ERR_ARG;
    *N = p->geom.N;
    return IWFPM_OK;
}

int iwfpm_grid_shape(iwfpm_plan_t p, int32_t* ext) {
    if (!p || !ext) return IWFPM_ERR_ARG;
    for (int ax = 0; ax < p->n; ++ax) ext[ax] = p->geom.ext[ax];
    return IWFPM_OK;
}

int iwfpm_indices(iwfpm_plan_t p, int32_t* k_out) {
    if (!p || !k_out) return IWFPM_ERR_ARG;
    std::vector<int> k(p->n);
    for (long long gp = 0; gp < p->geom.N; ++gp) {
        host_label(p, gp, k.data());
        long long vp = host_grid_to_vec(p, gp);
        for (int j = 0; j < p->n; ++j) k_out[vp * p->n + j] = k[j];
    }
    return IWFPM_OK;
}

int iwfpm_kinetic(iwfpm_plan_t p, double* out) {
    if (!p || !out) return IWFPM_ERR_ARG;
    std::vector<int> k(p->n);
    for (long long gp = 0; gp < p->geom.N; ++gp) {
        host_label(p, gp, k.data());
        out[host_grid_to_vec(p, gp)] = host_kinetic(p, k.data());
    }
    return IWFPM_OK;
}

int iwfpm_norm_bound(iwfpm_plan_t p, double* out) {
    if (!p || !out) return IWFPM_ERR_ARG;
    *out = p->lam_max + p->vsum_abs;
    return IWFPM_OK;
}

int iwfpm_apply_prec(iwfpm_plan_t p, const void* psi, void* hpsi, int nvec, int precision, void* stream) {
    if (!p || nvec < 0) return IWFPM_ERR_ARG;
    if (precision != IWFPM_PREC_FP64 && precision != IWFPM_PREC_FP32) return IWFPM_ERR_ARG;
    if (nvec > 0 && (!psi || !hpsi)) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    if (nvec == 0) return IWFPM_OK;
    const char* a = (const char*)psi;
    const char* b = (const char*)hpsi;
    size_t bytes = (size_t)nvec * (size_t)p->geom.N * 16;
    if (a < b + bytes && b < a + bytes) return IWFPM_ERR_ARG;  // overlapping buffers
    DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    return plan_apply(p, psi, hpsi, nvec, precision, (hipStream_t)stream);
}

int iwfpm_conv(iwfpm_plan_t p, const void* psi, void* out, int nvec, int precision, void* stream) {
    if (!p || nvec < 0) return IWFPM_ERR_ARG;
    if (precision != IWFPM_PREC_FP64 && precision != IWFPM_PREC_FP32) return IWFPM_ERR_ARG;
    if (nvec > 0 && (!psi || !out)) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    if (nvec == 0) return IWFPM_OK;
    const char* a = (const char*)psi;
    const char* b = (const char*)out;
    size_t bytes = (size_t)nvec * (size_t)p->geom.N * 16;
    if (a < b + bytes && b < a + bytes) return IWFPM_ERR_ARG;
    DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    return plan_apply(p, psi, out, nvec, precision, (hipStream_t)stream, 0);
}

int iwfpm_profile(iwfpm_plan_t p, int enable) {
    if (!p) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    DeviceGuard guard(p->opts.device);
    ApplyProfiler& pr = p->prof;
    for (auto& s : pr.ring) prof_collect(s, pr);
    if (enable) {
        if (pr.ring.empty()) {
            pr.ring.resize(1024);
            for (auto& s : pr.ring)
                for (auto& e : s.ev)
                    if (hipEventCreate(&e) != hipSuccess) return IWFPM_ERR_DEVICE;
        }
        for (int k = 0; k < 4; ++k) {
            pr.ms[k] = 0.0;
            pr.launches[k] = 0;
            pr.points[k] = 0;
        }
    }
    pr.on = enable != 0;
    return IWFPM_OK;
}

int iwfpm_profile_read(iwfpm_plan_t p, double* ms, int64_t* launches, int64_t* points) {
    if (!p || !ms || !launches || !points) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    DeviceGuard guard(p->opts.device);
    for (auto& s : p->prof.ring) prof_collect(s, p->prof);
    for (int k = 0; k < 4; ++k) {
        ms[k] = p->prof.ms[k];
        launches[k] = p->prof.launches[k];
        points[k] = p->prof.points[k];
    }
    return IWFPM_OK;
}

static std::string tune_key(const iwfpm_plan_s* p, int prec, int nvec) {
    std::string k = "prec=" + std::to_string(prec) + ";order=" + std::to_string(p->opts.order) +
                    ";vmode=" + std::to_string(p->geom.vmode) + ";d=" + std::to_string(p->d) +
                    ";nvec=" + std::to_string(nvec) + ";ext=";
    for (int ax = 0; ax < p->n; ++ax) k += std::to_string(p->geom.ext[ax]) + (ax + 1 < p->n ? "x" : "");
    return k;
}

static bool tune_cache_lookup(const char* path, const std::string& key, Schedule& sc, const iwfpm_plan_s* p,
                              int prec) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[512];
        int fused, split, tile, G, threads = 0;
        double us = 0.0;
        if (std::sscanf(line, "%511s %d %d %d %d %lf %d", k, &fused, &split, &tile, &G, &us, &threads) < 5) continue;
        if (key != k) continue;
        if (fused) {
            found = false;  // re-derive below
            sc.fused = true;
            found = true;
        } else {
            Schedule c{};
            c.pd.split = split;
            c.pd.s_in = p->geom.stride[split - 1];
            c.pd.s_out = p->geom.N / c.pd.s_in;
            c.pd.tile = tile;
            c.pd.slabs_per_wg = G;
            c.pd.xcd_remap = 1;
            finalize_threepass(p, c, prec, threads);
            sc = c;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

int iwfpm_tune(iwfpm_plan_t p, int nvec, int precision, void* stream, double* best_us) {
    if (!p || nvec < 1) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    const int prec = precision < 0 ? p->opts.precision : (precision == IWFPM_PREC_FP32 ? 1 : 0);
    DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    std::vector<Schedule> cands = schedule_candidates(p, prec);
    if (cands.empty()) return IWFPM_ERR_UNSUPPORTED;
    if (cands.size() == 1 && !cands[0].fused && cands[0].pd.split_mid > 0) {
        p->sched[prec] = cands[0];  // the one five-pass schedule: nothing to choose
        if (best_us) *best_us = -1.0;
        return IWFPM_OK;
    }
    const std::string key = tune_key(p, prec, nvec);
    const char* cache = std::getenv("IWFPM_TUNE_CACHE");
    if (cache && cache[0]) {
        Schedule sc{};
        if (tune_cache_lookup(cache, key, sc, p, prec)) {
            if (sc.fused) {
                for (auto& c : cands)
                    if (c.fused) sc = c;
            }
            if (sc.ok) {
                p->sched[prec] = sc;
                if (best_us) *best_us = -1.0;
                return IWFPM_OK;
            }
        }
    }
    DeviceBuf x, y;
    const size_t bytes = (size_t)nvec * p->geom.N * 16;
    if (dev_alloc(x, bytes) != IWFPM_OK || dev_alloc(y, bytes) != IWFPM_OK) {
        dev_free(x);
        dev_free(y);
        return IWFPM_ERR_ALLOC;
    }
    if (hipMemsetAsync(x.ptr, 0, bytes, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const Schedule keep = p->sched[prec];
    const bool prof = p->prof.on;
    p->prof.on = false;
    double best = 1e300;
    Schedule best_sc = keep;
    int rc = IWFPM_OK;
    for (const Schedule& c : cands) {
        p->sched[prec] = c;
        if ((rc = plan_apply(p, x.ptr, y.ptr, nvec, prec, st)) != IWFPM_OK) break;
        (void)hipEventRecord(e0, st);
        const int reps = 3;
        for (int r = 0; r < reps && rc == IWFPM_OK; ++r) rc = plan_apply(p, x.ptr, y.ptr, nvec, prec, st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) rc = IWFPM_ERR_DEVICE;
        if (rc != IWFPM_OK) break;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        double us = 1e3 * ms / reps;
        if (us < best) {
            best = us;
            best_sc = c;
        }
    }
    p->prof.on = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dev_free(x);
    dev_free(y);
    if (rc != IWFPM_OK) {
        p->sched[prec] = keep;
        return rc;
    }
    p->sched[prec] = best_sc;
    if (best_us) *best_us = best;
    if (cache && cache[0]) {
        if (FILE* f = std::fopen(cache, "a")) {
            std::fprintf(f, "%s %d %d %d %d %.3f %d\n", key.c_str(), best_sc.fused ? 1 : 0, best_sc.pd.split,
                         best_sc.pd.tile, best_sc.pd.slabs_per_wg, best, best_sc.pd.threads_outer);
            std::fclose(f);
        }
    }
    return IWFPM_OK;
}

int iwfpm_schedule(iwfpm_plan_t p, int precision, int32_t* out) {
    if (!p || !out) return IWFPM_ERR_ARG;
    const int prec = precision < 0 ? p->opts.precision : (precision == IWFPM_PREC_FP32 ? 1 : 0);
    const Schedule& sc = p->sched[prec];
    if (!sc.ok) return IWFPM_ERR_UNSUPPORTED;
    out[0] = sc.fused ? 1 : 0;
    out[1] = sc.pd.split;
    out[2] = sc.pd.tile;
    out[3] = sc.pd.slabs_per_wg;
    out[4] = sc.fused ? sc.threads_fused : sc.pd.threads_outer;
    return IWFPM_OK;
}

int iwfpm_apply(iwfpm_plan_t p, const void* psi, void* hpsi, int nvec, void* stream) {
    if (!p) return IWFPM_ERR_ARG;
    return iwfpm_apply_prec(p, psi, hpsi, nvec, p->opts.precision, stream);
}

}  // extern "C"
