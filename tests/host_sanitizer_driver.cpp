// Host-only exercise of libiwfpm's C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (tests/test_host_sanitizers.py).
// No GPU is touched: plans are host-only (device = -1), and the dense
// Rayleigh-Ritz solvers run on the host.  Every call's result is checked for
// the invariants that need no reference (shapes, ranges, residuals,
// orthonormality), and each error path must come back as its status code.
// Exit status 0 means every check passed and no sanitizer reported.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "iwfpm.h"

using cd = std::complex<double>;

static int g_fail = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            ++g_fail;                                     \
        }                                                 \
    } while (0)

// deterministic uniform numbers in [-1, 1)
static uint64_t g_state = 0x2404045070ull;
static double urand() {
    g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

struct Problem {
    int d, n;
    std::vector<double> P;  // d x n row-major
    std::vector<int32_t> K, L;
    std::vector<int32_t> modes;  // n_modes x n
    std::vector<double> vhat;    // n_modes x (re, im)
};

// const + sum_j w cos(y_j): Vhat_{+-e_j} = w / 2
static void cosine_modes(Problem& p, double w, double c) {
    const int n = p.n;
    if (c != 0.0) {
        for (int a = 0; a < n; ++a) p.modes.push_back(0);
        p.vhat.push_back(c);
        p.vhat.push_back(0.0);
    }
    for (int j = 0; j < n; ++j)
        for (int s : {1, -1}) {
            for (int a = 0; a < n; ++a) p.modes.push_back(a == j ? s : 0);
            p.vhat.push_back(w / 2.0);
            p.vhat.push_back(0.0);
        }
}

static Problem problem_1d(int K, int L) {
    Problem p{1, 2, {1.0, 0.5 * (std::sqrt(5.0) - 1.0)}, {K}, {L}, {}, {}};
    cosine_modes(p, 1.0, 0.0);
    return p;
}

static Problem problem_2d(int K, int L) {
    const double c = std::cos(M_PI / 6.0), s = std::sin(M_PI / 6.0);
    Problem p{2, 4, {1.0, 0.0, c, -s, 0.0, 1.0, s, c}, {K, K}, {L, L}, {}, {}};
    cosine_modes(p, 0.5, 0.0);
    return p;
}

static Problem problem_3d(double beta, int K, int L) {
    const double c = std::cos(0.2 * M_PI), s = std::sin(0.2 * M_PI), f = beta / (2.0 * M_PI);
    const double a = 0.5 * (std::sqrt(5.0) - 1.0);
    Problem p{3, 6, {f, 0, 0, f * c, -f * s, 0, 0, f, 0, f * s, f * c, 0, 0, 0, f, 0, 0, f * a}, {K, K, K}, {L, L, L},
              {}, {}};
    cosine_modes(p, -1.0, 6.0);
    return p;
}

static int make_plan(const Problem& p, int window, int order, iwfpm_plan_t* out) {
    iwfpm_opts o;
    iwfpm_default_opts(&o);
    o.device = -1;
    o.window_variant = window;
    o.order = order;
    return iwfpm_plan(p.d, p.n, p.P.data(), p.K.data(), p.L.data(), (int)p.vhat.size() / 2, p.modes.data(),
                      p.vhat.data(), &o, out);
}

static void check_plan(const Problem& p, int window, int order) {
    iwfpm_plan_t h = nullptr;
    int st = make_plan(p, window, order, &h);
    CHECK(st == IWFPM_OK && h, "plan d=%d n=%d window=%d order=%d: %s", p.d, p.n, window, order,
          iwfpm_status_string(st));
    if (st != IWFPM_OK) return;
    int64_t N = 0;
    CHECK(iwfpm_dof(h, &N) == IWFPM_OK, "dof");
    std::vector<int32_t> ext(p.n);
    CHECK(iwfpm_grid_shape(h, ext.data()) == IWFPM_OK, "grid_shape");
    int64_t prod = 1;
    for (int a = 0; a < p.n; ++a) prod *= ext[a];
    CHECK(prod == N, "N = %lld, product of extents %lld", (long long)N, (long long)prod);
    std::vector<int32_t> k((size_t)N * p.n);
    CHECK(iwfpm_indices(h, k.data()) == IWFPM_OK, "indices");
    // every label of the trailing (k_II) axes lies in [-L, L)
    for (int64_t i = 0; i < N; ++i)
        for (int j = 0; j < p.n - p.d; ++j) {
            const int32_t v = k[(size_t)i * p.n + p.d + j];
            if (v < -p.L[j] || v >= p.L[j]) {
                CHECK(false, "label %d of entry %lld outside [-L, L)", v, (long long)i);
                i = N;
                break;
            }
        }
    std::vector<double> lam((size_t)N);
    CHECK(iwfpm_kinetic(h, lam.data()) == IWFPM_OK, "kinetic");
    double lmax = 0.0;
    for (double v : lam) {
        CHECK(std::isfinite(v) && v >= 0.0, "kinetic entry %g", v);
        lmax = std::fmax(lmax, v);
    }
    double nb = 0.0;
    CHECK(iwfpm_norm_bound(h, &nb) == IWFPM_OK && nb >= lmax, "norm bound %g below max kinetic %g", nb, lmax);
    // device entry points on a host-only plan are refused, not run
    CHECK(iwfpm_apply(h, nullptr, nullptr, 1, nullptr) == IWFPM_ERR_NODEVICE ||
              iwfpm_apply(h, nullptr, nullptr, 1, nullptr) == IWFPM_ERR_ARG,
          "apply on a host-only plan");
    int32_t sched[8] = {0};
    (void)iwfpm_schedule(h, IWFPM_PREC_FP64, sched);
    CHECK(iwfpm_destroy(h) == IWFPM_OK, "destroy");
}

static void check_plan_errors() {
    Problem p = problem_2d(3, 4);
    iwfpm_plan_t h = nullptr;
    iwfpm_opts o;
    iwfpm_default_opts(&o);
    o.device = -1;
    const int nm = (int)p.vhat.size() / 2;
    CHECK(iwfpm_plan(0, 4, p.P.data(), p.K.data(), p.L.data(), nm, p.modes.data(), p.vhat.data(), &o, &h) ==
              IWFPM_ERR_ARG, "d = 0");
    CHECK(iwfpm_plan(2, 2, p.P.data(), p.K.data(), p.L.data(), nm, p.modes.data(), p.vhat.data(), &o, &h) ==
              IWFPM_ERR_ARG, "n = d");
    CHECK(iwfpm_plan(2, 4, p.P.data(), p.K.data(), p.L.data(), nm, p.modes.data(), p.vhat.data(), &o, nullptr) ==
              IWFPM_ERR_ARG, "NULL out");
    CHECK(iwfpm_plan(2, 4, nullptr, p.K.data(), p.L.data(), nm, p.modes.data(), p.vhat.data(), &o, &h) ==
              IWFPM_ERR_ARG, "NULL P");
    std::vector<int32_t> K0{0, 3};
    CHECK(iwfpm_plan(2, 4, p.P.data(), K0.data(), p.L.data(), nm, p.modes.data(), p.vhat.data(), &o, &h) ==
              IWFPM_ERR_ARG, "K = 0");
    std::vector<double> Pn = p.P;
    Pn[3] = NAN;
    CHECK(iwfpm_plan(2, 4, Pn.data(), p.K.data(), p.L.data(), nm, p.modes.data(), p.vhat.data(), &o, &h) ==
              IWFPM_ERR_ARG, "non-finite P");
    std::vector<double> Ps = p.P;  // P_I singular: its first two columns equal
    Ps[1] = Ps[0];
    Ps[5] = Ps[4];
    CHECK(iwfpm_plan(2, 4, Ps.data(), p.K.data(), p.L.data(), nm, p.modes.data(), p.vhat.data(), &o, &h) ==
              IWFPM_ERR_SINGULAR_PI, "singular P_I");
    std::vector<double> vh = p.vhat;  // Vhat_{e_1} != conj(Vhat_{-e_1}): not a real potential
    vh[1] = 0.25;
    CHECK(iwfpm_plan(2, 4, p.P.data(), p.K.data(), p.L.data(), nm, p.modes.data(), vh.data(), &o, &h) ==
              IWFPM_ERR_NONHERMITIAN, "non-Hermitian modes");
    std::vector<int32_t> K17{17, 17};  // a 34-point axis has no transform
    const int st = iwfpm_plan(2, 4, p.P.data(), K17.data(), p.L.data(), nm, p.modes.data(), p.vhat.data(), &o, &h);
    CHECK(st == IWFPM_ERR_UNSUPPORTED || st == IWFPM_OK, "2K = 34: %s", iwfpm_status_string(st));
    if (st == IWFPM_OK) iwfpm_destroy(h);
    for (int s = -12; s <= 1; ++s) CHECK(iwfpm_status_string(s) != nullptr, "status string %d", s);
    int64_t N;
    CHECK(iwfpm_dof(nullptr, &N) == IWFPM_ERR_ARG, "dof(NULL)");
    CHECK(iwfpm_destroy(nullptr) == IWFPM_ERR_ARG || iwfpm_destroy(nullptr) == IWFPM_OK, "destroy(NULL)");
}

// random Hermitian matrix (column-major), with an optional cluster of equal
// eigenvalues: A = Q diag(ev) Q^H for a unitary Q from Gram-Schmidt
static std::vector<cd> hermitian(int n, int cluster, bool real) {
    std::vector<cd> Q((size_t)n * n);
    for (auto& q : Q) q = cd(urand(), real ? 0.0 : urand());
    for (int j = 0; j < n; ++j) {
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                cd s = 0.0;
                for (int r = 0; r < n; ++r) s += std::conj(Q[r + (size_t)i * n]) * Q[r + (size_t)j * n];
                for (int r = 0; r < n; ++r) Q[r + (size_t)j * n] -= s * Q[r + (size_t)i * n];
            }
        double nr = 0.0;
        for (int r = 0; r < n; ++r) nr += std::norm(Q[r + (size_t)j * n]);
        for (int r = 0; r < n; ++r) Q[r + (size_t)j * n] /= std::sqrt(nr);
    }
    std::vector<double> ev(n);
    for (int i = 0; i < n; ++i) ev[i] = i < cluster ? -1.0 : 3.0 * urand();
    std::vector<cd> A((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            cd s = 0.0;
            for (int k = 0; k < n; ++k) s += Q[i + (size_t)k * n] * ev[k] * std::conj(Q[j + (size_t)k * n]);
            A[i + (size_t)j * n] = s;
        }
    for (int j = 0; j < n; ++j) {
        A[j + (size_t)j * n] = A[j + (size_t)j * n].real();
        for (int i = j + 1; i < n; ++i) A[j + (size_t)i * n] = std::conj(A[i + (size_t)j * n]);
    }
    return A;
}

// max over columns of ||A v - w v|| and of |V^H V - I|
static void pair_errors(const std::vector<cd>& A, int n, const double* w, const std::vector<cd>& V, int nv,
                        double* res, double* orth) {
    *res = 0.0;
    *orth = 0.0;
    for (int c = 0; c < nv; ++c) {
        double r2 = 0.0;
        for (int i = 0; i < n; ++i) {
            cd s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i + (size_t)k * n] * V[k + (size_t)c * n];
            r2 += std::norm(s - w[c] * V[i + (size_t)c * n]);
        }
        *res = std::fmax(*res, std::sqrt(r2));
        for (int c2 = 0; c2 < nv; ++c2) {
            cd s = 0.0;
            for (int k = 0; k < n; ++k) s += std::conj(V[k + (size_t)c2 * n]) * V[k + (size_t)c * n];
            *orth = std::fmax(*orth, std::abs(s - (c == c2 ? 1.0 : 0.0)));
        }
    }
}

static void check_dense() {
    for (int n : {1, 2, 5, 17, 40, 60, 96})
        for (int cluster : {0, 3})
            for (bool real : {true, false}) {
                if (cluster > n) continue;
                std::vector<cd> A = hermitian(n, cluster, real);
                for (int nv : {0, 1, n / 3, n}) {
                    std::vector<double> w(n);
                    std::vector<cd> V((size_t)n * std::max(nv, 1));
                    const int st = iwfpm_dense_heev_lowest(n, nv, reinterpret_cast<const double*>(A.data()), w.data(),
                                                           reinterpret_cast<double*>(V.data()));
                    CHECK(st == IWFPM_OK, "heev_lowest n=%d nv=%d: %s", n, nv, iwfpm_status_string(st));
                    for (int i = 1; i < n; ++i) CHECK(w[i - 1] <= w[i], "heev_lowest: eigenvalues not ascending");
                    double res, orth;
                    pair_errors(A, n, w.data(), V, nv, &res, &orth);
                    CHECK(res <= 1e-12 * n && orth <= 1e-12 * n, "heev_lowest n=%d nv=%d res %g orth %g", n, nv, res,
                          orth);
                }
                // A c = w B c with B = I + (a positive semidefinite part)
                std::vector<cd> B = hermitian(n, 0, real);
                for (int j = 0; j < n; ++j) {
                    for (int i = 0; i < n; ++i) B[i + (size_t)j * n] *= 0.1;
                    B[j + (size_t)j * n] += 1.0;
                }
                std::vector<double> w(n);
                std::vector<cd> C((size_t)n * n);
                CHECK(iwfpm_dense_geneig(n, reinterpret_cast<const double*>(A.data()),
                                         reinterpret_cast<const double*>(B.data()), w.data(),
                                         reinterpret_cast<double*>(C.data())) == IWFPM_OK,
                      "geneig n=%d", n);
                CHECK(iwfpm_dense_geneig(n, reinterpret_cast<const double*>(A.data()), nullptr, w.data(),
                                         reinterpret_cast<double*>(C.data())) == IWFPM_OK,
                      "geneig (B = I) n=%d", n);
                double res, orth;
                pair_errors(A, n, w.data(), C, n, &res, &orth);
                CHECK(res <= 1e-12 * n && orth <= 1e-12 * n, "geneig n=%d res %g orth %g", n, res, orth);
                // SVQB of a rank-deficient Gram matrix: G = M^H M with M of rank n / 2
                const int rk = std::max(1, n / 2);
                std::vector<cd> M((size_t)n * n, 0.0), G((size_t)n * n, 0.0), T((size_t)n * n);
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i)
                        M[i + (size_t)j * n] = j < rk ? cd(urand(), real ? 0.0 : urand()) : M[i + (size_t)(j - rk) * n];
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) {
                        cd s = 0.0;
                        for (int k = 0; k < n; ++k) s += std::conj(M[k + (size_t)i * n]) * M[k + (size_t)j * n];
                        G[i + (size_t)j * n] = s;
                    }
                int rank = -1;
                CHECK(iwfpm_dense_svqb(n, reinterpret_cast<const double*>(G.data()), reinterpret_cast<double*>(T.data()),
                                       &rank) == IWFPM_OK,
                      "svqb n=%d", n);
                CHECK(rank == rk, "svqb n=%d rank %d, expected %d", n, rank, rk);
            }
    std::vector<double> w(4), V(8);
    CHECK(iwfpm_dense_heev_lowest(0, 0, V.data(), w.data(), V.data()) == IWFPM_ERR_ARG, "heev_lowest n = 0");
    CHECK(iwfpm_dense_heev_lowest(2, 3, V.data(), w.data(), V.data()) == IWFPM_ERR_ARG, "heev_lowest nv > n");
    int rank;
    CHECK(iwfpm_dense_svqb(0, V.data(), V.data(), &rank) == IWFPM_ERR_ARG, "svqb k = 0");
}

int main() {
    const Problem probs[] = {problem_1d(8, 16), problem_1d(5, 60), problem_2d(3, 4), problem_2d(6, 20),
                             problem_3d(M_PI, 2, 3), problem_3d(0.5 * M_PI, 3, 2)};
    for (const Problem& p : probs)
        for (int window : {IWFPM_WINDOW_EXACT, IWFPM_WINDOW_ROUNDED, IWFPM_WINDOW_PM})
            for (int order : {IWFPM_ORDER_GRID, IWFPM_ORDER_WINDOW}) check_plan(p, window, order);
    check_plan_errors();
    check_dense();
    if (g_fail) {
        std::fprintf(stderr, "%d check(s) failed\n", g_fail);
        return 1;
    }
    std::printf("host sanitizer driver: all checks passed\n");
    return 0;
}
