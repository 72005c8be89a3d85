// learned.cpp - learned preconditioner: network, per-plan state, training.
//
// The preconditioner (formula and features in iwfpm.h) starts from the
// diagonal M of eq:precond (Sec. 4.1) and learns, per kinetic-energy shell,
// a rescaling of M plus the weights of two spectral-convolution layers built
// on the plan's own potential convolution C = F V F^{-1}.  Everything grid
// sized runs on the GPU (learned_kernels.hip and the apply's convolution);
// the host only builds the shell map and features once per plan, draws the
// initial weights and solves the small Rayleigh-Ritz problems of the loss.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <random>
#include <vector>

#include "learned.hpp"
#include "learned_dev.hpp"
#include "plan.hpp"

namespace iwfpm {

constexpr int kFeat = IWFPM_LEARNED_FEATURES;
constexpr int kHid = IWFPM_LEARNED_HIDDEN;
constexpr int kLayers = 4;

}  // namespace iwfpm

struct iwfpm_learned_s {
    int device = 0;
    int S = 1024;
    uint64_t seed = 0;
    int in[iwfpm::kLayers], out[iwfpm::kLayers];
    size_t offw[iwfpm::kLayers], offb[iwfpm::kLayers], offbeta = 0, np = 0;
    iwfpm::DeviceBuf w32, wbf, am, av, g;  // masters, bfloat16 copies, Adam moments, gradient
    long long version = 1;                  // bumped on every weight change
    long long t = 0;                        // Adam steps taken
    std::vector<iwfpm::LearnedPrecond*> users;
};

namespace iwfpm {

struct LearnedPrecond {
    iwfpm_learned_s* net = nullptr;
    iwfpm_plan_s* plan = nullptr;
    int S = 0;
    long long N = 0;
    int conv_prec = 0;
    std::vector<int> h_shell;
    std::vector<float> h_feat;
    DeviceBuf shell, feat, M, D0, E;
    DeviceBuf act;    // Z1 Y1 Z2 Y2 Z3 Y3 (S x H each), O (S x 2)
    DeviceBuf bwd;    // two S x H scratch arrays, dO as float (S x 2)
    DeviceBuf red;    // dO (S x 2 double), dbeta (3), flag
    DeviceBuf work;   // wblocks blocks of wcols columns
    DeviceBuf small, partial;  // Gram results / coefficients, Gram partial sums (training)
    int wcols = 0, wblocks = 0;
    long long version = 0;
};

static size_t red_doubles(int S) { return (size_t)2 * S + 3 + 1; }

static void net_layout(iwfpm_learned_s* n) {
    const int dims[kLayers + 1] = {kFeat, kHid, kHid, kHid, 2};
    size_t off = 0;
    for (int l = 0; l < kLayers; ++l) {
        n->in[l] = dims[l];
        n->out[l] = dims[l + 1];
        n->offw[l] = off;
        off += (size_t)dims[l] * dims[l + 1];
        n->offb[l] = off;
        off += dims[l + 1];
    }
    n->offbeta = off;
    n->np = off + 2;
}

static int upload_params(iwfpm_learned_s* n, const float* h, hipStream_t st) {
    if (hipMemcpyAsync(n->w32.ptr, h, n->np * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    if (lp_to_bf16((const float*)n->w32.ptr, (uint16_t*)n->wbf.ptr, (int)n->np, st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    if (hipMemsetAsync(n->am.ptr, 0, n->np * sizeof(float), st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if (hipMemsetAsync(n->av.ptr, 0, n->np * sizeof(float), st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return IWFPM_ERR_DEVICE;
    n->t = 0;
    ++n->version;
    return IWFPM_OK;
}

// ---------------------------------------------------------------------------
// per-plan state
// ---------------------------------------------------------------------------

static void lp_release(LearnedPrecond* lp) {
    dev_free(lp->shell);
    dev_free(lp->feat);
    dev_free(lp->M);
    dev_free(lp->D0);
    dev_free(lp->E);
    dev_free(lp->act);
    dev_free(lp->bwd);
    dev_free(lp->red);
    dev_free(lp->work);
    dev_free(lp->small);
    dev_free(lp->partial);
    lp->wcols = lp->wblocks = 0;
}

static void detach(LearnedPrecond* lp) {
    if (!lp->net) return;
    auto& u = lp->net->users;
    u.erase(std::remove(u.begin(), u.end(), lp), u.end());
    lp->net = nullptr;
}

// shell map and features of the plan (formulas in iwfpm.h)
static void shells_and_features(const iwfpm_plan_s* p, int S, std::vector<int>& shell, std::vector<float>& feat) {
    const long long N = p->geom.N;
    std::vector<double> e(N);
    std::vector<int> k(p->n);
    double emax = 0.0;
    for (long long gp = 0; gp < N; ++gp) {
        host_label(p, gp, k.data());
        double v = host_kinetic(p, k.data());
        e[host_grid_to_vec(p, gp)] = v;
        emax = std::max(emax, v);
    }
    shell.assign(N, 0);
    if (emax > 0.0)
        for (long long i = 0; i < N; ++i) {
            double t = std::floor((double)S * std::sqrt(e[i] / emax));
            shell[i] = t >= S - 1 ? S - 1 : (int)t;
        }
    double nu = p->vsum_nonzero, v0 = p->vhat0, sigma = std::max(0.0, nu - v0), S2 = 0.0;
    for (size_t i = 0; i < p->vre.size(); ++i) {
        bool zero = true;
        for (int j = 0; j < p->n; ++j) zero = zero && p->modes[i * p->n + j] == 0;
        if (!zero) S2 += p->vre[i] * p->vre[i] + p->vim[i] * p->vim[i];
    }
    auto ratio = [](double a, double b) { return b > 0.0 ? a / b : 0.0; };
    feat.assign((size_t)S * kFeat, 0.f);
    for (int s = 0; s < S; ++s) {
        double c = (s + 0.5) / S, es = emax * c * c, h = es + v0 + sigma;
        float* f = &feat[(size_t)s * kFeat];
        f[0] = (float)c;
        f[1] = (float)(std::log1p(es) / 8.0);
        f[2] = (float)ratio(es, es + nu);
        f[3] = (float)(std::log1p(nu) / 4.0);
        f[4] = (float)ratio(h * h, h * h + S2);
        f[5] = (float)ratio(nu, h);
        f[6] = (float)(std::log1p(emax) / 8.0);
        f[7] = (float)ratio(std::sqrt(es), std::sqrt(es) + std::sqrt(nu));
    }
}

static int lp_build(LearnedPrecond* lp, iwfpm_plan_s* p, int S) {
    lp->plan = p;
    lp->S = S;
    lp->N = p->geom.N;
    int prec = p->opts.precision == IWFPM_PREC_FP32 ? 1 : 0;
    lp->conv_prec = p->sched[prec].ok ? prec : 1 - prec;
    shells_and_features(p, S, lp->h_shell, lp->h_feat);
    std::vector<double> M;
    precond_diagonal(p, M);
    const long long N = lp->N;
    if (dev_alloc(lp->shell, N * sizeof(int)) || dev_alloc(lp->feat, (size_t)S * kFeat * sizeof(float)) ||
        dev_alloc(lp->M, N * sizeof(double)) || dev_alloc(lp->D0, N * sizeof(double)) ||
        dev_alloc(lp->E, N * sizeof(double)) ||
        dev_alloc(lp->act, ((size_t)6 * S * kHid + 2 * S) * sizeof(float)) ||
        dev_alloc(lp->bwd, ((size_t)2 * S * kHid + 2 * S) * sizeof(float)) ||
        dev_alloc(lp->red, red_doubles(S) * sizeof(double)))
        return IWFPM_ERR_ALLOC;
    if (hipMemcpy(lp->shell.ptr, lp->h_shell.data(), N * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(lp->feat.ptr, lp->h_feat.data(), lp->h_feat.size() * sizeof(float), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(lp->M.ptr, M.data(), N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    lp->version = 0;
    return IWFPM_OK;
}

static float* act_at(LearnedPrecond* lp, int i) { return (float*)lp->act.ptr + (size_t)i * lp->S * kHid; }
static float* out_o(LearnedPrecond* lp) { return act_at(lp, 6); }
static double* red_dO(LearnedPrecond* lp) { return (double*)lp->red.ptr; }
static double* red_dbeta(LearnedPrecond* lp) { return (double*)lp->red.ptr + 2 * lp->S; }
static int* red_flag(LearnedPrecond* lp) { return (int*)(red_dbeta(lp) + 3); }

// MLP over the shells and D0, E on the grid, when the weights changed
static int lp_forward_mlp(LearnedPrecond* lp, hipStream_t st) {
    iwfpm_learned_s* n = lp->net;
    if (!n) return IWFPM_ERR_WEIGHTS;
    if (lp->version == n->version) return IWFPM_OK;
    const int S = lp->S;
    const float* x = (const float*)lp->feat.ptr;
    const float* w32 = (const float*)n->w32.ptr;
    const uint16_t* wbf = (const uint16_t*)n->wbf.ptr;
    for (int l = 0; l < kLayers; ++l) {
        bool last = l == kLayers - 1;
        float* Z = last ? nullptr : act_at(lp, 2 * l);
        float* Y = last ? out_o(lp) : act_at(lp, 2 * l + 1);
        if (lp_dense_fwd(x, wbf + n->offw[l], w32 + n->offb[l], Z, Y, S, n->in[l], n->out[l], last ? 0 : 1, st) !=
            hipSuccess)
            return IWFPM_ERR_DEVICE;
        x = Y;
    }
    // weights that overflow the scalings are refused (the solver then uses M)
    if (lp_expand((const double*)lp->M.ptr, (const int*)lp->shell.ptr, out_o(lp), (double*)lp->D0.ptr,
                  (double*)lp->E.ptr, lp->N, st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    int* flag = red_flag(lp);
    if (hipMemsetAsync(flag, 0, sizeof(int), st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if (lp_nonfinite(w32 + n->offbeta, 2, flag, st) != hipSuccess ||
        lp_nonfinite_d((const double*)lp->D0.ptr, lp->N, flag, st) != hipSuccess ||
        lp_nonfinite_d((const double*)lp->E.ptr, lp->N, flag, st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    int h = 0;
    if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if (h) return IWFPM_ERR_WEIGHTS;
    lp->version = n->version;
    return IWFPM_OK;
}

// work blocks (wcols columns each): the first three serve the forward pass,
// the rest the training loss
enum { WB_TMP, WB_A, WB_C, WB_W, WB_G, WB_B1, WB_B2, WB_HX, WB_Y, WB_HY, WB_R, WB_HW, WB_COUNT };
constexpr int kGramBlocks = 512;

static int lp_ensure_work(LearnedPrecond* lp, int m, int blocks) {
    if (lp->wcols >= m && lp->wblocks >= blocks) return IWFPM_OK;
    int cols = std::max(m, lp->wcols), nb = std::max(blocks, lp->wblocks);
    if (dev_alloc(lp->work, (size_t)nb * cols * lp->N * sizeof(double2))) {
        lp->wcols = lp->wblocks = 0;
        return IWFPM_ERR_ALLOC;
    }
    lp->wcols = cols;
    lp->wblocks = nb;
    return IWFPM_OK;
}

static double2* wblock(LearnedPrecond* lp, int b) { return (double2*)lp->work.ptr + (size_t)b * lp->wcols * lp->N; }

static int conv(LearnedPrecond* lp, const double2* in, double2* out, int m, hipStream_t st) {
    return plan_apply(lp->plan, in, out, m, lp->conv_prec, st, 0);
}

// A = C(E R), Cc = C(E A) and W = (D0 + b1 a^2 E) R + E (2 a b1 A + b1 Cc); R, W as column pointers
static int lp_forward(LearnedPrecond* lp, const ColPtrs& R, const ColPtrs& W, int m, double2* A, double2* Cc,
                      hipStream_t st) {
    int rc = lp_forward_mlp(lp, st);
    if (rc) return rc;
    const double* D0 = (const double*)lp->D0.ptr;
    const double* E = (const double*)lp->E.ptr;
    double2* tmp = wblock(lp, WB_TMP);
    if (lp_scale_cols(R, tmp, m, E, lp->N, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if ((rc = conv(lp, tmp, A, m, st))) return rc;
    if (lp_scale(A, tmp, m, E, lp->N, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if ((rc = conv(lp, tmp, Cc, m, st))) return rc;
    const float* beta = (const float*)lp->net->w32.ptr + lp->net->offbeta;
    if (lp_combine(R, A, Cc, W, m, D0, E, beta, lp->N, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    return IWFPM_OK;
}

static ColPtrs contiguous_cols(const double2* base, int m, long long N) {
    ColPtrs c{};
    for (int j = 0; j < m; ++j) c.p[j] = const_cast<double2*>(base) + (size_t)j * N;
    return c;
}

using cvec = std::vector<std::complex<double>>;

// out (p x q, column-major) = L^H R
static int dgram(LearnedPrecond* lp, const ColPtrs& L, int p, const ColPtrs& R, int q, cvec& out, hipStream_t st) {
    double2* dC = (double2*)lp->small.ptr;
    if (gram(L, p, R, q, lp->N, (double2*)lp->partial.ptr, kGramBlocks, dC, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    out.assign((size_t)p * q, 0.0);
    if (hipMemcpyAsync(out.data(), dC, out.size() * sizeof(double2), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    return IWFPM_OK;
}

// Y_j = beta Y_j + sum_i A_i C[i + j p]
static int dlincomb(LearnedPrecond* lp, const ColPtrs& A, int p, const ColPtrs& Y, int q, const cvec& C, double beta,
                    hipStream_t st) {
    double2* dC = (double2*)lp->small.ptr + kMaxCols * kMaxCols;
    if (hipMemcpyAsync(dC, C.data(), (size_t)p * q * sizeof(double2), hipMemcpyHostToDevice, st) != hipSuccess ||
        lincomb(A, p, Y, q, dC, beta, lp->N, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    return IWFPM_OK;
}

static void hermitize(cvec& A, int k) {
    for (int j = 0; j < k; ++j) {
        A[j + (size_t)j * k] = A[j + (size_t)j * k].real();
        for (int i = 0; i < j; ++i) {
            std::complex<double> a = 0.5 * (A[i + (size_t)j * k] + std::conj(A[j + (size_t)i * k]));
            A[i + (size_t)j * k] = a;
            A[j + (size_t)i * k] = std::conj(a);
        }
    }
}

// Rayleigh-Ritz of (A, B) (k x k; B a Gram matrix): Ritz values ascending and
// C (k x r) with C^H B C = I; returns r (numerically dependent directions dropped)
static int small_rr(const cvec& A, const cvec& B, int k, std::vector<double>& th, cvec& C) {
    cvec T;
    const int r = svqb(B, k, T, 1e-12);
    if (r == 0) return 0;
    cvec AT((size_t)k * r, 0.0), A2((size_t)r * r, 0.0);
    for (int j = 0; j < r; ++j)
        for (int l = 0; l < k; ++l) {
            const std::complex<double> t = T[l + (size_t)j * k];
            for (int i = 0; i < k; ++i) AT[i + (size_t)j * k] += A[i + (size_t)l * k] * t;
        }
    for (int j = 0; j < r; ++j)
        for (int i = 0; i < r; ++i) {
            std::complex<double> acc = 0.0;
            for (int l = 0; l < k; ++l) acc += std::conj(T[l + (size_t)i * k]) * AT[l + (size_t)j * k];
            A2[i + (size_t)j * r] = acc;
        }
    hermitize(A2, r);
    cvec V;
    heev(A2, r, th, V);
    C.assign((size_t)k * r, 0.0);
    for (int j = 0; j < r; ++j)
        for (int l = 0; l < r; ++l) {
            const std::complex<double> v = V[l + (size_t)j * r];
            for (int i = 0; i < k; ++i) C[i + (size_t)j * k] += T[i + (size_t)l * k] * v;
        }
    return r;
}

// gradient of the loss in net->g from G = dL/dW (W = T(R)); A = C(E R), Cc = C(E A)
static int lp_backprop(LearnedPrecond* lp, const double2* G, const double2* R, const double2* A, const double2* Cc,
                       int m, hipStream_t st) {
    iwfpm_learned_s* n = lp->net;
    const long long N = lp->N;
    double2 *B1 = wblock(lp, WB_B1), *B2 = wblock(lp, WB_B2), *tmp = wblock(lp, WB_TMP);
    // adjoint convolutions: B1 = C(E G), B2 = C(E B1)   (C is Hermitian)
    const double* E = (const double*)lp->E.ptr;
    int rc;
    if (lp_scale(G, tmp, m, E, N, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if ((rc = conv(lp, tmp, B1, m, st))) return rc;
    if (lp_scale(B1, tmp, m, E, N, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if ((rc = conv(lp, tmp, B2, m, st))) return rc;
    const int S = lp->S;
    if (hipMemsetAsync(red_dO(lp), 0, (2 * S + 3) * sizeof(double), st) != hipSuccess) return IWFPM_ERR_DEVICE;
    const float* beta = (const float*)n->w32.ptr + n->offbeta;
    if (lp_shell_grad(G, R, A, Cc, B1, B2, m, (const double*)lp->M.ptr, (const double*)lp->D0.ptr, E, beta,
                      (const int*)lp->shell.ptr, red_dO(lp), red_dbeta(lp), N, st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    // back through the MLP
    float* g = (float*)n->g.ptr;
    const uint16_t* wbf = (const uint16_t*)n->wbf.ptr;
    float* dcur = (float*)lp->bwd.ptr + (size_t)2 * S * kHid;  // dO as float, S x 2
    float* s0 = (float*)lp->bwd.ptr;
    float* s1 = s0 + (size_t)S * kHid;
    if (lp_to_float(red_dO(lp), dcur, 2 * S, 1.0, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if (lp_beta_grad(red_dbeta(lp), beta, g + n->offbeta, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    for (int l = kLayers - 1; l >= 0; --l) {
        const float* X = l == 0 ? (const float*)lp->feat.ptr : act_at(lp, 2 * (l - 1) + 1);
        float* dX = l == 0 ? nullptr : (dcur == s0 ? s1 : s0);
        if (lp_dense_bwd(X, dcur, wbf + n->offw[l], dX, g + n->offw[l], g + n->offb[l], S, n->in[l], n->out[l], st) !=
            hipSuccess)
            return IWFPM_ERR_DEVICE;
        if (l > 0) {
            // dZ_{l-1} = dY_{l-1} .* GELU'(Z_{l-1}), in place
            if (lp_act_bwd(dX, act_at(lp, 2 * (l - 1)), dX, S * kHid, 1, st) != hipSuccess) return IWFPM_ERR_DEVICE;
            dcur = dX;
        }
    }
    return IWFPM_OK;
}

// Training loss of one iterate block X (m columns) with the exact lowest
// eigenvalues lam: the share of eigenvalue error left after one
// Rayleigh-Ritz step on [Y, T(R)],
//   Y, theta = Ritz pairs of span(X),  R = H Y - Y theta,  W = T(R),
//   theta' = lowest m Ritz values of span([Y W]),
//   loss = sum_j (theta'_j - lam_j) / sum_j (theta_j - lam_j).
// With S = [Y W], HS = H S and C' the B-orthonormal Ritz coefficients, the
// derivative of theta'_j with respect to W (as d/dRe + i d/dIm) is
// 2 (HS c'_j - theta'_j S c'_j) c'_{W,j}^H, which gives G below.  H is applied
// in float64 whenever the plan has a float64 schedule.
static int lp_rr_loss_grad(LearnedPrecond* lp, const double2* X, int m, const double* lam, bool grad, double* loss,
                           int* nvalid, hipStream_t st) {
    *nvalid = 0;
    *loss = 0.0;
    if (m < 1 || 2 * m > kMaxCols) return IWFPM_ERR_ARG;
    int rc = lp_ensure_work(lp, m, WB_COUNT);
    if (rc) return rc;
    if (!lp->small.ptr && dev_alloc(lp->small, (size_t)2 * kMaxCols * kMaxCols * sizeof(double2)))
        return IWFPM_ERR_ALLOC;
    if (!lp->partial.ptr && dev_alloc(lp->partial, (size_t)kGramBlocks * kMaxCols * kMaxCols * sizeof(double2)))
        return IWFPM_ERR_ALLOC;
    iwfpm_plan_s* p = lp->plan;
    const long long N = lp->N;
    const int hprec = p->sched[0].ok ? 0 : 1;
    double2 *HX = wblock(lp, WB_HX), *Y = wblock(lp, WB_Y), *HY = wblock(lp, WB_HY), *R = wblock(lp, WB_R),
            *W = wblock(lp, WB_W), *HW = wblock(lp, WB_HW), *G = wblock(lp, WB_G), *A = wblock(lp, WB_A),
            *Cc = wblock(lp, WB_C);
    ColPtrs Xc = contiguous_cols(X, m, N), HXc = contiguous_cols(HX, m, N), Yc = contiguous_cols(Y, m, N),
            HYc = contiguous_cols(HY, m, N), Rc = contiguous_cols(R, m, N), Wc = contiguous_cols(W, m, N),
            Gc = contiguous_cols(G, m, N);
    if ((rc = plan_apply(p, X, HX, m, hprec, st, 1))) return rc;
    cvec Am, Bm, C;
    if ((rc = dgram(lp, Xc, m, HXc, m, Am, st)) || (rc = dgram(lp, Xc, m, Xc, m, Bm, st))) return rc;
    hermitize(Am, m);
    std::vector<double> th;
    if (small_rr(Am, Bm, m, th, C) < m) return IWFPM_OK;  // dependent block: no sample
    double D = 0.0;
    for (int j = 0; j < m; ++j) D += th[j] - lam[j];
    const double hn = p->lam_max + p->vsum_abs;
    if (!(D > 1e-12 * m * hn)) return IWFPM_OK;  // already converged: no sample
    if ((rc = dlincomb(lp, Xc, m, Yc, m, C, 0.0, st)) || (rc = dlincomb(lp, HXc, m, HYc, m, C, 0.0, st))) return rc;
    Reals t{};
    for (int j = 0; j < m; ++j) t.v[j] = th[j];
    if (residual(HYc, Yc, Rc, t, m, N, st) != hipSuccess) return IWFPM_ERR_DEVICE;
    if ((rc = lp_forward(lp, Rc, Wc, m, A, Cc, st))) return rc;
    if ((rc = plan_apply(p, W, HW, m, hprec, st, 1))) return rc;
    const int k = 2 * m;
    ColPtrs S{}, HS{};
    for (int j = 0; j < m; ++j) {
        S.p[j] = Yc.p[j];
        S.p[m + j] = Wc.p[j];
        HS.p[j] = HYc.p[j];
        HS.p[m + j] = HW + (size_t)j * N;
    }
    cvec A2, B2, C2;
    if ((rc = dgram(lp, S, k, HS, k, A2, st)) || (rc = dgram(lp, S, k, S, k, B2, st))) return rc;
    hermitize(A2, k);
    std::vector<double> th2;
    const int r2 = small_rr(A2, B2, k, th2, C2);
    if (r2 < m) return IWFPM_OK;
    double num = 0.0;
    for (int j = 0; j < m; ++j) num += th2[j] - lam[j];
    *loss = num / D;
    *nvalid = 1;
    if (!std::isfinite(*loss)) return IWFPM_ERR_NUMERIC;
    if (!grad) return IWFPM_OK;
    // G = HS P1 - S P2, P1 = (2/D) C'_m C'_{W,m}^H, P2 = (2/D) C'_m diag(theta'_m) C'_{W,m}^H
    cvec P1((size_t)k * m, 0.0), P2((size_t)k * m, 0.0);
    for (int l = 0; l < m; ++l)
        for (int j = 0; j < m; ++j) {
            const std::complex<double> cw = std::conj(C2[(m + l) + (size_t)j * k]) * (2.0 / D);
            for (int i = 0; i < k; ++i) {
                const std::complex<double> v = C2[i + (size_t)j * k] * cw;
                P1[i + (size_t)l * k] += v;
                P2[i + (size_t)l * k] -= v * th2[j];
            }
        }
    if ((rc = dlincomb(lp, HS, k, Gc, m, P1, 0.0, st)) || (rc = dlincomb(lp, S, k, Gc, m, P2, 1.0, st))) return rc;
    return lp_backprop(lp, G, R, A, Cc, m, st);
}

static int net_adam(iwfpm_learned_s* n, double lr, hipStream_t st) {
    LearnedPrecond* any = n->users.empty() ? nullptr : n->users.front();
    int* flag = any ? red_flag(any) : nullptr;
    if (flag) {
        int h = 0;
        if (hipMemsetAsync(flag, 0, sizeof(int), st) != hipSuccess) return IWFPM_ERR_DEVICE;
        if (lp_nonfinite((const float*)n->g.ptr, (int)n->np, flag, st) != hipSuccess) return IWFPM_ERR_DEVICE;
        if (hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return IWFPM_ERR_DEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return IWFPM_ERR_DEVICE;
        if (h) return IWFPM_ERR_NUMERIC;
    }
    const float b1 = 0.9f, b2 = 0.999f;
    ++n->t;
    float c1 = 1.f - std::pow(b1, (float)n->t), c2 = 1.f - std::pow(b2, (float)n->t);
    if (lp_adam((float*)n->w32.ptr, (float*)n->am.ptr, (float*)n->av.ptr, (const float*)n->g.ptr,
                (uint16_t*)n->wbf.ptr, (int)n->np, (float)lr, b1, b2, c1, c2, 1e-8f, st) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    ++n->version;
    return IWFPM_OK;
}

static int lp_step(LearnedPrecond* lp, const double2* X, int m, const double* lam, double lr, double* loss,
                   int* used, hipStream_t st) {
    int nv = 0;
    int rc = lp_rr_loss_grad(lp, X, m, lam, true, loss, &nv, st);
    if (used) *used = nv;
    if (rc) return rc;
    if (nv == 0) return IWFPM_OK;
    return net_adam(lp->net, lr, st);
}

// ---------------------------------------------------------------------------
// hooks used by the eigensolver
// ---------------------------------------------------------------------------

bool learned_ready(const LearnedPrecond* lp, const iwfpm_plan_s* p) {
    return lp && lp->net && lp->plan == p && lp->N == p->geom.N;
}

int learned_apply(LearnedPrecond* lp, iwfpm_plan_s* p, const ColPtrs& R, const ColPtrs& W, int m, hipStream_t st) {
    if (!learned_ready(lp, p)) return IWFPM_ERR_WEIGHTS;
    if (m == 0) return IWFPM_OK;
    int rc = lp_ensure_work(lp, m, 3);
    if (rc) return rc;
    return lp_forward(lp, R, W, m, wblock(lp, WB_A), wblock(lp, WB_C), st);
}

void learned_free(LearnedPrecond* lp) {
    if (!lp) return;
    detach(lp);
    lp_release(lp);
    delete lp;
}

}  // namespace iwfpm

using namespace iwfpm;

static int attach(iwfpm_plan_t p, iwfpm_learned_t n) {
    if (p->learned && p->learned->net == n && learned_ready(p->learned, p)) return IWFPM_OK;
    if (!p->learned) p->learned = new LearnedPrecond();
    LearnedPrecond* lp = p->learned;
    detach(lp);
    if (!n) return IWFPM_OK;
    if (lp->S != n->S || lp->plan != p || lp->N != p->geom.N || !lp->shell.ptr) {
        lp_release(lp);
        int rc = lp_build(lp, p, n->S);
        if (rc) {
            lp_release(lp);
            lp->S = 0;
            return rc;
        }
    }
    lp->net = n;
    lp->version = 0;
    n->users.push_back(lp);
    return IWFPM_OK;
}

extern "C" {

void iwfpm_default_learned_opts(iwfpm_learned_opts* o) {
    if (!o) return;
    o->device = 0;
    o->shells = 1024;
    o->seed = 2404045070ull;
}

void iwfpm_default_train_opts(iwfpm_train_opts* o) {
    if (!o) return;
    o->steps = 3000;
    o->lr = 1e-3;
    o->nev = 8;
    o->block = 0;
    o->tol = 1e-8;
    o->maxit = 1000;
    o->snapshots = 24;
    o->stride = 4;
    o->seed = 2404045070ull;
}

int iwfpm_learned_create(const iwfpm_learned_opts* o, iwfpm_learned_t* out) {
    if (!o || !out) return IWFPM_ERR_ARG;
    *out = nullptr;
    if (o->shells < 1 || o->shells > 65536) return IWFPM_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || o->device < 0 || o->device >= ndev) return IWFPM_ERR_DEVICE;
    DeviceGuard guard(o->device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    auto* n = new iwfpm_learned_s();
    n->device = o->device;
    n->S = o->shells;
    n->seed = o->seed;
    net_layout(n);
    if (dev_alloc(n->w32, n->np * sizeof(float)) || dev_alloc(n->wbf, n->np * sizeof(uint16_t)) ||
        dev_alloc(n->am, n->np * sizeof(float)) || dev_alloc(n->av, n->np * sizeof(float)) ||
        dev_alloc(n->g, n->np * sizeof(float))) {
        iwfpm_learned_destroy(n);
        return IWFPM_ERR_ALLOC;
    }
    // hidden layers uniform in +-1/sqrt(fan_in); the output layer and beta start at
    // zero so that a new network reproduces M
    std::vector<float> h(n->np, 0.f);
    std::mt19937_64 rng(o->seed);
    for (int l = 0; l < kLayers - 1; ++l) {
        float bound = 1.f / std::sqrt((float)n->in[l]);
        std::uniform_real_distribution<float> u(-bound, bound);
        for (size_t i = 0; i < (size_t)n->in[l] * n->out[l]; ++i) h[n->offw[l] + i] = u(rng);
        for (int i = 0; i < n->out[l]; ++i) h[n->offb[l] + i] = u(rng);
    }
    int rc = upload_params(n, h.data(), nullptr);
    if (rc) {
        iwfpm_learned_destroy(n);
        return rc;
    }
    *out = n;
    return IWFPM_OK;
}

int iwfpm_learned_destroy(iwfpm_learned_t n) {
    if (!n) return IWFPM_ERR_ARG;
    DeviceGuard guard(n->device);
    (void)hipDeviceSynchronize();
    for (LearnedPrecond* lp : n->users) lp->net = nullptr;
    n->users.clear();
    dev_free(n->w32);
    dev_free(n->wbf);
    dev_free(n->am);
    dev_free(n->av);
    dev_free(n->g);
    delete n;
    return IWFPM_OK;
}

int iwfpm_learned_nparams(iwfpm_learned_t n, int64_t* np) {
    if (!n || !np) return IWFPM_ERR_ARG;
    *np = (int64_t)n->np;
    return IWFPM_OK;
}

int iwfpm_learned_get(iwfpm_learned_t n, float* params) {
    if (!n || !params) return IWFPM_ERR_ARG;
    DeviceGuard guard(n->device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return IWFPM_ERR_DEVICE;
    if (hipMemcpy(params, n->w32.ptr, n->np * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    return IWFPM_OK;
}

int iwfpm_learned_set(iwfpm_learned_t n, const float* params) {
    if (!n || !params) return IWFPM_ERR_ARG;
    for (size_t i = 0; i < n->np; ++i)
        if (!std::isfinite(params[i])) return IWFPM_ERR_WEIGHTS;
    DeviceGuard guard(n->device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return IWFPM_ERR_DEVICE;
    return upload_params(n, params, nullptr);
}

int iwfpm_learned_attach(iwfpm_plan_t p, iwfpm_learned_t n) {
    if (!p) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    if (n && n->device != p->opts.device) return IWFPM_ERR_ARG;
    DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    return attach(p, n);
}

int iwfpm_learned_shells(iwfpm_plan_t p, int32_t* shell, float* features) {
    if (!p) return IWFPM_ERR_ARG;
    LearnedPrecond* lp = p->learned;
    if (!lp || !lp->net) return IWFPM_ERR_WEIGHTS;
    if (shell) std::memcpy(shell, lp->h_shell.data(), lp->h_shell.size() * sizeof(int32_t));
    if (features) std::memcpy(features, lp->h_feat.data(), lp->h_feat.size() * sizeof(float));
    return IWFPM_OK;
}

static int check_block_args(iwfpm_plan_t p, const void* a, const void* b, int nvec) {
    if (!p || nvec < 1 || nvec > kMaxCols || !a || !b) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    if (!learned_ready(p->learned, p)) return IWFPM_ERR_WEIGHTS;
    return IWFPM_OK;
}

int iwfpm_learned_forward(iwfpm_plan_t p, const void* r, void* t, int nvec, void* stream) {
    int rc = check_block_args(p, r, t, nvec);
    if (rc) return rc;
    const char* a = (const char*)r;
    const char* b = (const char*)t;
    size_t bytes = (size_t)nvec * (size_t)p->geom.N * sizeof(double2);
    if (a < b + bytes && b < a + bytes) return IWFPM_ERR_ARG;
    DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    const long long N = p->geom.N;
    return learned_apply(p->learned, p, contiguous_cols((const double2*)r, nvec, N),
                         contiguous_cols((const double2*)t, nvec, N), nvec, (hipStream_t)stream);
}

int iwfpm_learned_grad(iwfpm_plan_t p, const void* x, int nvec, const double* lam, double* loss, float* grad,
                       void* stream) {
    if (!p || !x || !lam || !loss || nvec < 1 || 2 * nvec > kMaxCols) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    if (!learned_ready(p->learned, p)) return IWFPM_ERR_WEIGHTS;
    DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    LearnedPrecond* lp = p->learned;
    iwfpm_learned_s* n = lp->net;
    if (grad && hipMemsetAsync(n->g.ptr, 0, n->np * sizeof(float), st) != hipSuccess) return IWFPM_ERR_DEVICE;
    int nv = 0;
    int rc = lp_rr_loss_grad(lp, (const double2*)x, nvec, lam, grad != nullptr, loss, &nv, st);
    if (rc) return rc;
    if (grad) {
        if (hipMemcpyAsync(grad, n->g.ptr, n->np * sizeof(float), hipMemcpyDeviceToHost, st) != hipSuccess)
            return IWFPM_ERR_DEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return IWFPM_ERR_DEVICE;
    }
    return nv ? IWFPM_OK : IWFPM_ERR_NUMERIC;
}

int iwfpm_learned_step(iwfpm_plan_t p, const void* x, int nvec, const double* lam, double lr, double* loss,
                       void* stream) {
    if (!p || !x || !lam || !loss || nvec < 1 || 2 * nvec > kMaxCols || !(lr > 0.0)) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    if (!learned_ready(p->learned, p)) return IWFPM_ERR_WEIGHTS;
    DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    int used = 0;
    int rc = lp_step(p->learned, (const double2*)x, nvec, lam, lr, loss, &used, st);
    if (rc) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return IWFPM_ERR_DEVICE;
    return used ? IWFPM_OK : IWFPM_ERR_NUMERIC;
}

int iwfpm_learned_train(iwfpm_learned_t n, int B, const iwfpm_plan_t* plans, const iwfpm_train_opts* o, double* loss,
                        void* stream) {
    if (!n || B < 1 || !plans || !o) return IWFPM_ERR_ARG;
    if (o->steps < 0 || !(o->lr > 0.0) || o->nev < 1 || o->nev > kMaxCols || !(o->tol > 0.0) || o->maxit < 1 ||
        o->snapshots < 1 || o->snapshots > 64 || o->stride < 1)
        return IWFPM_ERR_ARG;
    for (int i = 0; i < B; ++i) {
        if (!plans[i]) return IWFPM_ERR_ARG;
        if (plans[i]->host_only) return IWFPM_ERR_NODEVICE;
        if (plans[i]->opts.device != n->device) return IWFPM_ERR_ARG;
        if (o->nev > plans[i]->geom.N) return IWFPM_ERR_ARG;
    }
    DeviceGuard guard(n->device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    hipStream_t st = (hipStream_t)stream;
    const int nev = o->nev;
    struct Sample {
        int plan;
        double2* X;
    };
    std::vector<DeviceBuf> store(B);
    std::vector<std::vector<double>> lam(B);
    std::vector<Sample> samples;
    int rc = IWFPM_OK;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        for (auto& b : store) dev_free(b);
    };
    for (int i = 0; i < B && rc == IWFPM_OK; ++i) {
        iwfpm_plan_t p = plans[i];
        if ((rc = attach(p, n))) break;
        const size_t blk = (size_t)nev * p->geom.N;
        if (dev_alloc(store[i], blk * o->snapshots * sizeof(double2))) {
            rc = IWFPM_ERR_ALLOC;
            break;
        }
        Capture cap;
        cap.stride = o->stride;
        cap.ncol = nev;
        for (int c = 0; c < o->snapshots; ++c) cap.X.push_back((double2*)store[i].ptr + (size_t)c * blk);
        iwfpm_eigs_opts eo;
        iwfpm_default_eigs_opts(&eo);
        eo.nev = nev;
        eo.block = o->block;
        eo.tol = o->tol;
        eo.maxit = o->maxit;
        eo.precond = IWFPM_PRECOND_PLAIN;
        eo.seed = o->seed + (uint64_t)i;
        lam[i].assign(nev, 0.0);
        int erc = eigs_capture(p, eo, &cap, lam[i].data(), nullptr, st);
        if (erc != IWFPM_OK && erc != IWFPM_ERR_NOCONV) {
            rc = erc;
            break;
        }
        // iterates whose columns were all converged carry no training signal
        for (int c = 0; c < cap.got; ++c) {
            double worst = 0.0;
            for (double e : cap.eta[c]) worst = std::max(worst, e);
            if (worst > 10.0 * o->tol) samples.push_back({i, cap.X[c]});
        }
    }
    if (rc == IWFPM_OK && samples.empty()) rc = IWFPM_ERR_NUMERIC;
    if (rc) {
        cleanup();
        return rc;
    }
    std::mt19937_64 rng(o->seed ^ 0x9e3779b97f4a7c15ull);
    std::uniform_int_distribution<size_t> pick(0, samples.size() - 1);
    for (int s = 0; s < o->steps; ++s) {
        const Sample& sm = samples[pick(rng)];
        double l = 0.0;
        int used = 0;
        int src = lp_step(plans[sm.plan]->learned, sm.X, nev, lam[sm.plan].data(), o->lr, &l, &used, st);
        if (src == IWFPM_ERR_NUMERIC || !used) l = std::nan("");
        else if (src) {
            rc = src;
            break;
        }
        if (loss) loss[s] = l;
    }
    cleanup();
    return rc;
}

}  // extern "C"
