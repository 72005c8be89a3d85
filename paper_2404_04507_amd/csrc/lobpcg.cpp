// lobpcg.cpp - iwfpm_eigs: block LOBPCG for the lowest eigenpairs of H~.
//
// The paper solves H~ U = E U with LOBPCG and the diagonal preconditioner of
// eq:precond (Sec. 4.1).  This is the block form: an orthonormal block X of
// m >= nev vectors, the preconditioned residuals W and the previous search
// directions P span the trial subspace of each Rayleigh-Ritz step.
//
//  * Every tall N x k operation runs on the GPU in float64 (blas_kernels.hip);
//    the apply runs in the plan's precision.  Only the small Gram matrices
//    (at most 96 x 96) come to the host, where the generalised eigenproblem is
//    solved by Cholesky + cyclic Jacobi (both written here).
//  * The trial basis [X W P] is kept orthonormal (so its Gram matrix is the
//    identity): W is orthogonalised against X and P twice and orthonormalised
//    by SVQB (scaled Gram eigen-decomposition, which drops numerically
//    dependent directions instead of failing); the next P is formed in the
//    small coefficient space, orthogonal to the new X, so no tall
//    orthogonalisation of P is needed.  X^H H X = diag(theta) is reused, so
//    only [X W P]^H [HW HP] is computed on the GPU.
//  * Soft locking: converged columns keep their place in X but contribute no
//    W and no P direction.
//  * Convergence: eta_i = ||H x_i - theta_i x_i|| / ((||H||_est + |theta_i|) ||x_i||)
//    with ||H||_est = max Lambda + sum |Vhat_m|.
//  * Float32-convolution plans iterate with float32 applies; convergence is
//    always confirmed by a final Rayleigh-Ritz with float64 applies, and when
//    float32 stalls (or the float64 check fails) the solver continues with
//    float64 applies (polish).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "blas.hpp"
#include "learned.hpp"
#include "plan.hpp"

using cd = std::complex<double>;

namespace iwfpm {

// ---------------------------------------------------------------------------
// small dense Hermitian linear algebra (column-major, A[i + j*n])
// ---------------------------------------------------------------------------

// A = L L^H, L lower triangular stored in A; false if A is not (numerically) PD
static bool cholesky(std::vector<cd>& A, int n) {
    double scale = 0.0;
    for (int i = 0; i < n; ++i) scale = std::max(scale, std::abs(A[i + i * n].real()));
    for (int j = 0; j < n; ++j) {
        double d = A[j + j * n].real();
        for (int k = 0; k < j; ++k) d -= std::norm(A[j + k * n]);
        if (!(d > 1e-13 * scale)) return false;
        double l = std::sqrt(d);
        A[j + j * n] = l;
        for (int i = j + 1; i < n; ++i) {
            cd s = A[i + j * n];
            for (int k = 0; k < j; ++k) s -= A[i + k * n] * std::conj(A[j + k * n]);
            A[i + j * n] = s / l;
        }
        for (int i = 0; i < j; ++i) A[i + j * n] = 0.0;
    }
    return true;
}

// cyclic Jacobi for Hermitian A: A = V diag(w) V^H, w ascending
static void jacobi_eigh(std::vector<cd> A, int n, std::vector<double>& w, std::vector<cd>& V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[i + i * n] = 1.0;
    double fro = 0.0;
    for (auto& a : A) fro += std::norm(a);
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < j; ++i) off += std::norm(A[i + j * n]);
        if (std::sqrt(off) <= 1e-17 * fro || fro == 0.0) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                cd apq = A[p + q * n];
                double g = std::abs(apq);
                if (g <= 1e-300) continue;
                double app = A[p + p * n].real(), aqq = A[q + q * n].real();
                // phase so that the (p, q) entry becomes real and positive
                cd ph = apq / g;  // e^{i phi}
                double tau = (aqq - app) / (2.0 * g);
                double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // J = diag(1, conj(ph)) * [[c, s], [-s, c]]
                cd j00 = c, j01 = s, j10 = -s * std::conj(ph), j11 = c * std::conj(ph);
                for (int k = 0; k < n; ++k) {  // columns: A J
                    cd akp = A[k + p * n], akq = A[k + q * n];
                    A[k + p * n] = akp * j00 + akq * j10;
                    A[k + q * n] = akp * j01 + akq * j11;
                }
                for (int k = 0; k < n; ++k) {  // rows: J^H A
                    cd apk = A[p + k * n], aqk = A[q + k * n];
                    A[p + k * n] = std::conj(j00) * apk + std::conj(j10) * aqk;
                    A[q + k * n] = std::conj(j01) * apk + std::conj(j11) * aqk;
                }
                A[p + q * n] = 0.0;
                A[q + p * n] = 0.0;
                A[p + p * n] = A[p + p * n].real();
                A[q + q * n] = A[q + q * n].real();
                for (int k = 0; k < n; ++k) {
                    cd vkp = V[k + p * n], vkq = V[k + q * n];
                    V[k + p * n] = vkp * j00 + vkq * j10;
                    V[k + q * n] = vkp * j01 + vkq * j11;
                }
            }
        }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::vector<double> d(n);
    for (int i = 0; i < n; ++i) d[i] = A[i + i * n].real();
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    std::vector<cd> Vs((size_t)n * n);
    w.resize(n);
    for (int j = 0; j < n; ++j) {
        w[j] = d[idx[j]];
        for (int i = 0; i < n; ++i) Vs[i + j * n] = V[i + idx[j] * n];
    }
    V.swap(Vs);
}

// sqrt(f^2 + g^2) without the cost of std::hypot when the squares can neither
// overflow nor underflow
static inline double pyth(double f, double g) {
    const double m = std::max(std::fabs(f), std::fabs(g));
    return (m > 1e-150 && m < 1e150) ? std::sqrt(f * f + g * g) : std::hypot(f, g);
}

// Hermitian eigen-decomposition A = V diag(w) V^H (w ascending) by Householder
// reduction to a real symmetric tridiagonal matrix followed by the implicit QL
// iteration with Wilkinson shifts; false if QL does not converge.  The QL
// sweep is the published tql2 procedure of Bowdler, Martin, Reinsch and
// Wilkinson (Numer. Math. 11, 1968; Handbook for Automatic Computation
// vol. II, contribution II/3; EISPACK's TQL2), with its usual roles of the
// shift g, the rotation pair (c, s) and the running values p, r, b.
static bool householder_ql(std::vector<cd> A, int n, std::vector<double>& w, std::vector<cd>& V) {
    // Q = H_0 H_1 ... accumulates the reflectors (column-major, column loops innermost)
    std::vector<cd> Q((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[i + (size_t)i * n] = 1.0;
    std::vector<cd> v(n), pv(n), acc(n);
    for (int k = 0; k + 2 < n; ++k) {
        // reflector H = I - 2 u u^H on rows/cols k+1..n-1 that zeroes A[k+2.., k]
        cd* ak = &A[(size_t)k * n];
        double xn = 0.0;
        for (int i = k + 1; i < n; ++i) xn += std::norm(ak[i]);
        xn = std::sqrt(xn);
        cd x0 = ak[k + 1];
        double tail = xn * xn - std::norm(x0);
        if (xn == 0.0 || tail <= 1e-300) continue;
        cd ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0);
        cd alpha = -ph * xn;
        double un = 0.0;
        for (int i = k + 1; i < n; ++i) {
            v[i] = ak[i];
            if (i == k + 1) v[i] -= alpha;
            un += std::norm(v[i]);
        }
        const double inv = 1.0 / std::sqrt(un);
        for (int i = k + 1; i < n; ++i) v[i] *= inv;
        v[k] = 0.0;
        // p = A u over rows k..n-1, K = u^H p, w = p - K u; A <- A - 2 (u w^H + w u^H)
        for (int i = k; i < n; ++i) pv[i] = 0.0;
        for (int j = k + 1; j < n; ++j) {
            const cd* aj = &A[(size_t)j * n];
            const cd vj = v[j];
            for (int i = k; i < n; ++i) pv[i] += aj[i] * vj;
        }
        cd K = 0.0;
        for (int i = k + 1; i < n; ++i) K += std::conj(v[i]) * pv[i];
        for (int i = k + 1; i < n; ++i) pv[i] -= K.real() * v[i];
        for (int j = k; j < n; ++j) {
            cd* aj = &A[(size_t)j * n];
            const cd a = 2.0 * std::conj(pv[j]), b = 2.0 * std::conj(v[j]);
            for (int i = k; i < n; ++i) aj[i] -= v[i] * a + pv[i] * b;
        }
        // Q <- Q H
        for (int r = 0; r < n; ++r) acc[r] = 0.0;
        for (int j = k + 1; j < n; ++j) {
            const cd* qj = &Q[(size_t)j * n];
            const cd vj = v[j];
            for (int r = 0; r < n; ++r) acc[r] += qj[r] * vj;
        }
        for (int j = k + 1; j < n; ++j) {
            cd* qj = &Q[(size_t)j * n];
            const cd c = 2.0 * std::conj(v[j]);
            for (int r = 0; r < n; ++r) qj[r] -= acc[r] * c;
        }
    }
    // real tridiagonal: d (diagonal), e (sub-diagonal made real by a diagonal phase
    // folded into the columns of Q)
    std::vector<double> d(n), e(n, 0.0);
    cd phase = 1.0;
    for (int k = 0; k < n; ++k) {
        d[k] = A[k + (size_t)k * n].real();
        if (k + 1 < n) {
            cd sub = A[(k + 1) + (size_t)k * n];
            double a = std::abs(sub);
            cd next = a > 0.0 ? phase * (sub / a) : phase;
            e[k] = a;
            for (int r = 0; r < n; ++r) Q[r + (size_t)(k + 1) * n] *= next;
            phase = next;
        }
    }
    // implicit QL with Wilkinson shifts (e[k] couples k and k+1); the rotations
    // act on the real matrix Z, and V = Q Z at the end
    std::vector<double> Z((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[i + (size_t)i * n] = 1.0;
    for (int l = 0; l < n; ++l) {
        int iter = 0, m;
        do {
            for (m = l; m < n - 1; ++m) {
                double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * dd) break;
            }
            if (m != l) {
                if (++iter > 80) return false;
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = pyth(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
                double sn = 1.0, cs = 1.0, pp = 0.0;
                int i;
                bool deflated = false;
                for (i = m - 1; i >= l; --i) {
                    double f = sn * e[i], b = cs * e[i];
                    r = pyth(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) {
                        d[i + 1] -= pp;
                        e[m] = 0.0;
                        deflated = true;
                        break;
                    }
                    sn = f / r;
                    cs = g / r;
                    g = d[i + 1] - pp;
                    r = (d[i] - g) * sn + 2.0 * cs * b;
                    pp = sn * r;
                    d[i + 1] = g + pp;
                    g = cs * r - b;
                    double* zi = &Z[(size_t)i * n];
                    double* zi1 = &Z[(size_t)(i + 1) * n];
                    for (int k = 0; k < n; ++k) {
                        const double fz = zi1[k];
                        zi1[k] = sn * zi[k] + cs * fz;
                        zi[k] = cs * zi[k] - sn * fz;
                    }
                }
                if (deflated) continue;
                d[l] -= pp;
                e[l] = g;
                e[m] = 0.0;
            }
        } while (m != l);
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    // V[:, j] = Q Z[:, idx[j]]
    V.assign((size_t)n * n, 0.0);
    w.resize(n);
    for (int j = 0; j < n; ++j) {
        w[j] = d[idx[j]];
        const double* zj = &Z[(size_t)idx[j] * n];
        cd* vj = &V[(size_t)j * n];
        for (int k = 0; k < n; ++k) {
            const double z = zj[k];
            if (z == 0.0) continue;
            const cd* qk = &Q[(size_t)k * n];
            for (int i = 0; i < n; ++i) vj[i] += qk[i] * z;
        }
    }
    return true;
}

// Householder reduction of a Hermitian matrix (lower triangle, column-major,
// split real/imaginary parts) to real symmetric tridiagonal form.  On exit:
// d (diagonal), sub (complex subdiagonal entries A[k+1][k]), and the
// reflectors u_k (unit, rows k+1..n-1) in columns of Ur/Ui with has[k].
static void tridiag_soa(std::vector<cd>& A, int n, std::vector<double>& d, std::vector<cd>& sub,
                        std::vector<double>& Ur, std::vector<double>& Ui, std::vector<char>& has) {
    std::vector<double> ar((size_t)n * n), ai((size_t)n * n);
    for (size_t e = 0; e < (size_t)n * n; ++e) {
        ar[e] = A[e].real();
        ai[e] = A[e].imag();
    }
    Ur.assign((size_t)n * n, 0.0);
    Ui.assign((size_t)n * n, 0.0);
    has.assign(n, 0);
    sub.assign(n, 0.0);
    d.assign(n, 0.0);
    std::vector<double> pr(n), pi(n);
    for (int k = 0; k + 2 < n; ++k) {
        const double* akr = &ar[(size_t)k * n];
        const double* aki = &ai[(size_t)k * n];
        double xn = 0.0;
        for (int i = k + 1; i < n; ++i) xn += akr[i] * akr[i] + aki[i] * aki[i];
        xn = std::sqrt(xn);
        const cd x0(akr[k + 1], aki[k + 1]);
        const double tail = xn * xn - std::norm(x0);
        if (xn == 0.0 || tail <= 1e-300) {
            sub[k] = x0;
            continue;
        }
        const cd ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0);
        const cd alpha = -ph * xn;
        double* ur = &Ur[(size_t)k * n];
        double* ui = &Ui[(size_t)k * n];
        double un = 0.0;
        for (int i = k + 1; i < n; ++i) {
            ur[i] = akr[i];
            ui[i] = aki[i];
        }
        ur[k + 1] -= alpha.real();
        ui[k + 1] -= alpha.imag();
        for (int i = k + 1; i < n; ++i) un += ur[i] * ur[i] + ui[i] * ui[i];
        const double inv = 1.0 / std::sqrt(un);
        for (int i = k + 1; i < n; ++i) {
            ur[i] *= inv;
            ui[i] *= inv;
        }
        has[k] = 1;
        sub[k] = alpha;
        // p = A22 u from the lower triangle: column j contributes A[i][j] u_j to
        // p_i (i > j) and conj(A[i][j]) u_i to p_j
        for (int i = k + 1; i < n; ++i) pr[i] = pi[i] = 0.0;
        for (int j = k + 1; j < n; ++j) {
            const double* ajr = &ar[(size_t)j * n];
            const double* aji = &ai[(size_t)j * n];
            const double ujr = ur[j], uji = ui[j];
            double s0r = 0, s0i = 0, s1r = 0, s1i = 0;
            int i = j + 1;
            for (; i + 1 < n; i += 2) {
                pr[i] += ajr[i] * ujr - aji[i] * uji;
                pi[i] += ajr[i] * uji + aji[i] * ujr;
                pr[i + 1] += ajr[i + 1] * ujr - aji[i + 1] * uji;
                pi[i + 1] += ajr[i + 1] * uji + aji[i + 1] * ujr;
                s0r += ajr[i] * ur[i] + aji[i] * ui[i];
                s0i += ajr[i] * ui[i] - aji[i] * ur[i];
                s1r += ajr[i + 1] * ur[i + 1] + aji[i + 1] * ui[i + 1];
                s1i += ajr[i + 1] * ui[i + 1] - aji[i + 1] * ur[i + 1];
            }
            for (; i < n; ++i) {
                pr[i] += ajr[i] * ujr - aji[i] * uji;
                pi[i] += ajr[i] * uji + aji[i] * ujr;
                s0r += ajr[i] * ur[i] + aji[i] * ui[i];
                s0i += ajr[i] * ui[i] - aji[i] * ur[i];
            }
            pr[j] += ajr[j] * ujr + s0r + s1r;
            pi[j] += ajr[j] * uji + s0i + s1i;
        }
        double K = 0.0;
        for (int i = k + 1; i < n; ++i) K += ur[i] * pr[i] + ui[i] * pi[i];
        for (int i = k + 1; i < n; ++i) {
            pr[i] -= K * ur[i];
            pi[i] -= K * ui[i];
        }
        // A22 <- A22 - 2 (u w^H + w u^H) on the lower triangle (w = p - K u)
        for (int j = k + 1; j < n; ++j) {
            double* ajr = &ar[(size_t)j * n];
            double* aji = &ai[(size_t)j * n];
            const double ar2 = 2.0 * pr[j], ai2 = -2.0 * pi[j];  // 2 conj(w_j)
            const double br2 = 2.0 * ur[j], bi2 = -2.0 * ui[j];  // 2 conj(u_j)
            for (int i = j; i < n; ++i) {
                ajr[i] -= ur[i] * ar2 - ui[i] * ai2 + pr[i] * br2 - pi[i] * bi2;
                aji[i] -= ur[i] * ai2 + ui[i] * ar2 + pr[i] * bi2 + pi[i] * br2;
            }
        }
    }
    if (n >= 2) sub[n - 2] = cd(ar[(size_t)(n - 1) + (size_t)(n - 2) * n], ai[(size_t)(n - 1) + (size_t)(n - 2) * n]);
    for (int k = 0; k < n; ++k) d[k] = ar[k + (size_t)k * n];
}

// Householder reduction of a real symmetric matrix (lower triangle,
// column-major) to tridiagonal form: d (diagonal), e (e[k] = T[k+1][k]) and
// the reflectors u_k (unit, rows k+1..n-1) in the columns of U with has[k].
static void tridiag_real(std::vector<double>& a, int n, std::vector<double>& d, std::vector<double>& e,
                         std::vector<double>& U, std::vector<char>& has) {
    // small dense algebra: sums may be reassociated (vectorised); the result
    // is still the same for every run of one build
#pragma clang fp reassociate(on)
    U.assign((size_t)n * n, 0.0);
    has.assign(n, 0);
    e.assign(n, 0.0);
    d.assign(n, 0.0);
    std::vector<double> p(n);
    for (int k = 0; k + 2 < n; ++k) {
        const double* ak = &a[(size_t)k * n];
        double xn = 0.0;
        for (int i = k + 1; i < n; ++i) xn += ak[i] * ak[i];
        xn = std::sqrt(xn);
        const double x0 = ak[k + 1];
        if (xn == 0.0 || xn * xn - x0 * x0 <= 1e-300) {
            e[k] = x0;
            continue;
        }
        const double alpha = x0 >= 0.0 ? -xn : xn;
        double* u = &U[(size_t)k * n];
        for (int i = k + 1; i < n; ++i) u[i] = ak[i];
        u[k + 1] -= alpha;
        double un = 0.0;
        for (int i = k + 1; i < n; ++i) un += u[i] * u[i];
        const double inv = 1.0 / std::sqrt(un);
        for (int i = k + 1; i < n; ++i) u[i] *= inv;
        has[k] = 1;
        e[k] = alpha;
        // p = A22 u from the lower triangle
        for (int i = k + 1; i < n; ++i) p[i] = 0.0;
        for (int j = k + 1; j < n; ++j) {
            const double* aj = &a[(size_t)j * n];
            const double uj = u[j];
            double s = 0.0;
            for (int i = j + 1; i < n; ++i) {
                p[i] += aj[i] * uj;
                s += aj[i] * u[i];
            }
            p[j] += aj[j] * uj + s;
        }
        double K = 0.0;
        for (int i = k + 1; i < n; ++i) K += u[i] * p[i];
        for (int i = k + 1; i < n; ++i) p[i] -= K * u[i];
        // A22 <- A22 - 2 (u w^T + w u^T) on the lower triangle (w = p - K u)
        for (int j = k + 1; j < n; ++j) {
            double* aj = &a[(size_t)j * n];
            const double pj = 2.0 * p[j], uj = 2.0 * u[j];
            for (int i = j; i < n; ++i) aj[i] -= u[i] * pj + p[i] * uj;
        }
    }
    if (n >= 2) e[n - 2] = a[(size_t)(n - 1) + (size_t)(n - 2) * n];
    for (int k = 0; k < n; ++k) d[k] = a[k + (size_t)k * n];
}

// Eigenvalues (all, ascending, in w) of the real symmetric tridiagonal matrix
// with diagonal d and off-diagonal e (e[k] couples k and k+1), and the
// eigenvectors of the nv lowest (Y: row-major n x nv).  Implicit QL with
// Wilkinson shifts on the eigenvalues alone, its plane rotations recorded;
// the selected eigenvectors are then rebuilt from unit vectors by the
// rotations in reverse order.  false if QL does not converge.
static bool tridiag_lowest(std::vector<double> d, std::vector<double> e, int n, int nv, std::vector<double>& w,
                           std::vector<double>& Y) {
    struct Rot {
        int i;
        double c, s;
    };
    std::vector<Rot> rots;
    rots.reserve((size_t)4 * n * n);
    for (int l = 0; l < n; ++l) {
        int iter = 0, m;
        do {
            for (m = l; m < n - 1; ++m) {
                double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * dd) break;
            }
            if (m != l) {
                if (++iter > 80) return false;
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = pyth(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
                double sn = 1.0, cs = 1.0, pp = 0.0;
                bool deflated = false;
                for (int i = m - 1; i >= l; --i) {
                    double f = sn * e[i], b = cs * e[i];
                    r = pyth(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) {
                        d[i + 1] -= pp;
                        e[m] = 0.0;
                        deflated = true;
                        break;
                    }
                    const double rinv = 1.0 / r;
                    sn = f * rinv;
                    cs = g * rinv;
                    g = d[i + 1] - pp;
                    r = (d[i] - g) * sn + 2.0 * cs * b;
                    pp = sn * r;
                    d[i + 1] = g + pp;
                    g = cs * r - b;
                    rots.push_back({i, cs, sn});
                }
                if (deflated) continue;
                d[l] -= pp;
                e[l] = g;
                e[m] = 0.0;
            }
        } while (m != l);
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    w.resize(n);
    for (int j = 0; j < n; ++j) w[j] = d[idx[j]];
    Y.assign((size_t)n * nv, 0.0);
    for (int c = 0; c < nv; ++c) Y[(size_t)idx[c] * nv + c] = 1.0;
    if (nv == 0) return true;  // eigenvalues only (Y is empty: no rows to rotate)
    for (size_t t = rots.size(); t-- > 0;) {
        const Rot& q = rots[t];
        double* __restrict yi = &Y[(size_t)q.i * nv];
        double* __restrict yi1 = yi + nv;
        const double qc = q.c, qs = q.s;
#pragma clang loop vectorize(enable)
        for (int c = 0; c < nv; ++c) {
            const double a = yi[c], b = yi1[c];
            yi[c] = qc * a + qs * b;
            yi1[c] = qc * b - qs * a;
        }
    }
    return true;
}

// Real symmetric eigenvalues (all, ascending) and the eigenvectors of the nv
// lowest (V: n x nv): tridiag_real, tridiag_lowest, then the reflectors in
// reverse order.
static bool syev_lowest(std::vector<double> A, int n, int nv, std::vector<double>& w, std::vector<double>& V) {
    // small dense algebra: sums may be reassociated (vectorised); the result
    // is still the same for every run of one build
#pragma clang fp reassociate(on)
    nv = std::max(0, std::min(nv, n));
    std::vector<double> d, e, U, Y;
    std::vector<char> has;
    tridiag_real(A, n, d, e, U, has);
    if (!tridiag_lowest(d, e, n, nv, w, Y)) return false;
    V.assign((size_t)n * nv, 0.0);
    for (int c = 0; c < nv; ++c)
        for (int i = 0; i < n; ++i) V[i + (size_t)c * n] = Y[(size_t)i * nv + c];
    for (int k = n - 3; k >= 0; --k) {
        if (!has[k]) continue;
        const double* u = &U[(size_t)k * n];
        for (int c = 0; c < nv; ++c) {
            double* vc = &V[(size_t)c * n];
            double s = 0.0;
            for (int i = k + 1; i < n; ++i) s += u[i] * vc[i];
            s *= 2.0;
            for (int i = k + 1; i < n; ++i) vc[i] -= u[i] * s;
        }
    }
    return true;
}

// true when every entry has an exactly zero imaginary part: the real-symmetric
// solver route produces such Hermitian matrices, and they are handed to the
// real arithmetic (the same results up to the order of rounding, at a
// quarter of the multiplications)
static bool exactly_real(const std::vector<cd>& A) {
    for (const cd& a : A)
        if (a.imag() != 0.0) return false;
    return true;
}

static std::vector<double> real_parts(const std::vector<cd>& A) {
    std::vector<double> r(A.size());
    for (size_t i = 0; i < A.size(); ++i) r[i] = A[i].real();
    return r;
}

static std::vector<cd> as_complex(const std::vector<double>& A) {
    return std::vector<cd>(A.begin(), A.end());
}

// Hermitian eigenvalues (all, ascending) and the eigenvectors of the nv
// lowest (V: n x nv), for the Rayleigh-Ritz step, which keeps only those.
// Householder reduction (tridiag_soa, the reflectors kept, not multiplied
// out), tridiag_lowest on the real tridiagonal matrix, then the diagonal
// phases and the reflectors in reverse order.  A matrix with exactly zero
// imaginary parts goes through syev_lowest.
static bool heev_lowest(std::vector<cd> A, int n, int nv, std::vector<double>& w, std::vector<cd>& V) {
    nv = std::max(0, std::min(nv, n));
    if (exactly_real(A)) {
        std::vector<double> Vr;
        if (!syev_lowest(real_parts(A), n, nv, w, Vr)) return false;
        V = as_complex(Vr);
        return true;
    }
    std::vector<double> d0, Ur, Ui;
    std::vector<cd> sub;
    std::vector<char> has;
    tridiag_soa(A, n, d0, sub, Ur, Ui, has);
    // real tridiagonal: d, and e made real by the diagonal phases ph
    std::vector<double> e(n, 0.0), Y;
    std::vector<cd> phs(n, 1.0);
    for (int k = 0; k + 1 < n; ++k) {
        const double a = std::abs(sub[k]);
        phs[k + 1] = a > 0.0 ? phs[k] * (sub[k] / a) : phs[k];
        e[k] = a;
    }
    if (!tridiag_lowest(d0, e, n, nv, w, Y)) return false;
    // V = H_0 ... H_{n-3} diag(ph) Y
    V.assign((size_t)n * nv, 0.0);
    for (int c = 0; c < nv; ++c) {
        cd* vc = &V[(size_t)c * n];
        for (int i = 0; i < n; ++i) vc[i] = phs[i] * Y[(size_t)i * nv + c];
    }
    for (int k = n - 3; k >= 0; --k) {
        if (!has[k]) continue;
        const double* ur = &Ur[(size_t)k * n];
        const double* ui = &Ui[(size_t)k * n];
        for (int c = 0; c < nv; ++c) {
            cd* vc = &V[(size_t)c * n];
            double sr = 0.0, si = 0.0;
            for (int i = k + 1; i < n; ++i) {
                sr += ur[i] * vc[i].real() + ui[i] * vc[i].imag();
                si += ur[i] * vc[i].imag() - ui[i] * vc[i].real();
            }
            sr *= 2.0;
            si *= 2.0;
            for (int i = k + 1; i < n; ++i) vc[i] -= cd(ur[i] * sr - ui[i] * si, ur[i] * si + ui[i] * sr);
        }
    }
    return true;
}

// Hermitian eigensolver used throughout: Householder + QL, Jacobi as fallback
void heev(const std::vector<cd>& A, int n, std::vector<double>& w, std::vector<cd>& V) {
    if (exactly_real(A)) {
        std::vector<double> Vr;
        if (syev_lowest(real_parts(A), n, n, w, Vr)) {
            V = as_complex(Vr);
            return;
        }
    }
    if (!householder_ql(A, n, w, V)) jacobi_eigh(A, n, w, V);
}

// The Rayleigh-Ritz and orthonormalisation algebra below is written once for
// complex (cd) and real (double) entries; the real-symmetric solver route
// hands exactly real matrices to the real instantiation.
static inline double conj_(double x) { return x; }
static inline cd conj_(const cd& x) { return std::conj(x); }
static inline double real_(double x) { return x; }
static inline double real_(const cd& x) { return x.real(); }

static void heev_t(const std::vector<cd>& A, int n, std::vector<double>& w, std::vector<cd>& V) { heev(A, n, w, V); }
static void heev_t(const std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V) {
    if (syev_lowest(A, n, n, w, V)) return;
    std::vector<cd> Vc;  // QL failed: the complex route (Jacobi as its fallback) keeps real data real
    heev(as_complex(A), n, w, Vc);
    V = real_parts(Vc);
}
static bool heev_lowest_t(const std::vector<cd>& A, int n, int nv, std::vector<double>& w, std::vector<cd>& V) {
    return heev_lowest(A, n, nv, w, V);
}
static bool heev_lowest_t(const std::vector<double>& A, int n, int nv, std::vector<double>& w,
                          std::vector<double>& V) {
    return syev_lowest(A, n, nv, w, V);
}

// SVQB: T (k x r) with (B T)^H (B T) = I for the Gram matrix G = B^H B (k x k);
// directions whose scaled eigenvalue is below eps are dropped.  Returns r.
template <class S>
static int svqb_t(const std::vector<S>& G, int k, std::vector<S>& T, double eps) {
    std::vector<double> dsc(k);
    for (int i = 0; i < k; ++i) {
        double g = real_(G[i + i * k]);
        dsc[i] = g > 0.0 ? 1.0 / std::sqrt(g) : 0.0;
    }
    std::vector<S> Sm((size_t)k * k);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i) Sm[i + j * k] = dsc[i] * G[i + j * k] * dsc[j];
    for (int j = 0; j < k; ++j)  // exact Hermitian symmetry
        for (int i = 0; i < j; ++i) {
            S a = 0.5 * (Sm[i + j * k] + conj_(Sm[j + i * k]));
            Sm[i + j * k] = a;
            Sm[j + i * k] = conj_(a);
        }
    std::vector<double> w;
    std::vector<S> U;
    heev_t(Sm, k, w, U);
    double wmax = k ? w[k - 1] : 0.0;
    std::vector<int> keep;
    for (int j = 0; j < k; ++j)
        if (w[j] > eps * wmax && w[j] > 0.0) keep.push_back(j);
    int r = (int)keep.size();
    T.assign((size_t)k * r, 0.0);
    for (int c = 0; c < r; ++c) {
        int j = keep[c];
        double f = 1.0 / std::sqrt(w[j]);
        for (int i = 0; i < k; ++i) T[i + c * k] = dsc[i] * U[i + j * k] * f;
    }
    return r;
}

int svqb(const std::vector<cd>& G, int k, std::vector<cd>& T, double eps) {
    if (exactly_real(G)) {
        std::vector<double> Tr;
        const int r = svqb_t(real_parts(G), k, Tr, eps);
        T = as_complex(Tr);
        return r;
    }
    return svqb_t(G, k, T, eps);
}

// A c = theta B c (Hermitian A, Hermitian PD B): theta ascending, C (n x n)
static bool gen_eigh(const std::vector<cd>& A, const std::vector<cd>& B, int n, std::vector<double>& theta,
                     std::vector<cd>& C) {
    std::vector<cd> L = B;
    if (!cholesky(L, n)) return false;
    // Z = L^{-1} A
    std::vector<cd> Z = A;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            cd s = Z[i + j * n];
            for (int k = 0; k < i; ++k) s -= L[i + k * n] * Z[k + j * n];
            Z[i + j * n] = s / L[i + i * n];
        }
    // At = L^{-1} Z^H
    std::vector<cd> At((size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            cd s = std::conj(Z[j + i * n]);
            for (int k = 0; k < i; ++k) s -= L[i + k * n] * At[k + j * n];
            At[i + j * n] = s / L[i + i * n];
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < j; ++i) {
            cd a = 0.5 * (At[i + j * n] + std::conj(At[j + i * n]));
            At[i + j * n] = a;
            At[j + i * n] = std::conj(a);
        }
    std::vector<cd> Y;
    heev(At, n, theta, Y);
    // C = L^{-H} Y
    C.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j)
        for (int i = n - 1; i >= 0; --i) {
            cd s = Y[i + j * n];
            for (int k = i + 1; k < n; ++k) s -= std::conj(L[k + i * n]) * C[k + j * n];
            C[i + j * n] = s / L[i + i * n].real();
        }
    return true;
}

// ---------------------------------------------------------------------------
// solver state
// ---------------------------------------------------------------------------

enum { B_X, B_HX, B_XN, B_HXN, B_P, B_HP, B_PN, B_HPN, B_W, B_HW, B_T1, B_COUNT };

// staging for small coefficient matrices sent to the device: a ring of
// pinned host slots, so that enqueueing never waits on the previous copy
constexpr int kRingSlots = 64;
constexpr size_t kSlot = (size_t)kMaxCols * 48;  // complex entries per slot

struct Solver {
    long long N = 0;
    int mcap = 0;
    DeviceBuf buf[B_COUNT];
    DeviceBuf M;          // preconditioner diagonal
    int Mkind = -1;
    DeviceBuf partial;    // gram / norm partials
    DeviceBuf dring;      // coefficient slots on the device
    double2* hsmall = nullptr;  // gram results and norms: pinned host memory the reductions write directly
    double2* hring = nullptr;   // pinned coefficient slots
    int ring_next = 0;
    int ring_since_sync = 0;
    int max_blocks = 1024;
};

static void solver_free(Solver* s) {
    if (!s) return;
    for (auto& b : s->buf) dev_free(b);
    dev_free(s->M);
    dev_free(s->partial);
    dev_free(s->dring);
    if (s->hsmall) (void)hipHostFree(s->hsmall);
    if (s->hring) (void)hipHostFree(s->hring);
    delete s;
}

static int solver_ensure(iwfpm_plan_s* p, int m) {
    Solver* s = (Solver*)p->solver;
    if (!s) {
        s = new Solver();
        p->solver = s;
    }
    s->N = p->geom.N;
    if (s->mcap < m) {
        for (auto& b : s->buf)
            if (dev_alloc(b, (size_t)s->N * m * sizeof(double2)) != IWFPM_OK) return IWFPM_ERR_ALLOC;
        s->mcap = m;
    }
    size_t need_partial = (size_t)s->max_blocks * kMaxCols * kMaxCols * sizeof(double2);
    if (s->partial.bytes < need_partial && dev_alloc(s->partial, need_partial) != IWFPM_OK) return IWFPM_ERR_ALLOC;
    size_t need_small = (size_t)2 * 96 * 96 * sizeof(double2);
    size_t need_ring = (size_t)kRingSlots * kSlot * sizeof(double2);
    if (s->dring.bytes < need_ring && dev_alloc(s->dring, need_ring) != IWFPM_OK) return IWFPM_ERR_ALLOC;
    if (!s->hsmall && hipHostMalloc((void**)&s->hsmall, need_small) != hipSuccess) return IWFPM_ERR_ALLOC;
    if (!s->hring && hipHostMalloc((void**)&s->hring, need_ring) != hipSuccess) return IWFPM_ERR_ALLOC;
    return IWFPM_OK;
}

// diagonal of eq:precond for H~ + sigma I (closed form for non-aliasing modes)
void precond_diagonal(const iwfpm_plan_s* p, std::vector<double>& M) {
    const long long N = p->geom.N;
    M.assign(N, 1.0);
    double sigma = std::max(0.0, p->vsum_nonzero - p->vhat0);
    double S = 0.0;
    const int n = p->n;
    for (size_t i = 0; i < p->vre.size(); ++i) {
        bool zero = true;
        for (int j = 0; j < n; ++j) zero = zero && p->modes[i * n + j] == 0;
        if (!zero) S += p->vre[i] * p->vre[i] + p->vim[i] * p->vim[i];
    }
    std::vector<int> k(n);
    for (long long gp = 0; gp < N; ++gp) {
        host_label(p, gp, k.data());
        double h = host_kinetic(p, k.data()) + p->vhat0 + sigma;
        M[host_grid_to_vec(p, gp)] = h / (h * h + S);
    }
}

static int solver_precond(iwfpm_plan_s* p, int kind) {
    Solver* s = (Solver*)p->solver;
    if (s->Mkind == kind && s->M.ptr) return IWFPM_OK;
    const long long N = p->geom.N;
    std::vector<double> M(N, 1.0);
    if (kind == IWFPM_PRECOND_PLAIN) precond_diagonal(p, M);
    if (dev_alloc(s->M, N * sizeof(double)) != IWFPM_OK) return IWFPM_ERR_ALLOC;
    if (hipMemcpy(s->M.ptr, M.data(), N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return IWFPM_ERR_DEVICE;
    s->Mkind = kind;
    return IWFPM_OK;
}

struct Ctx {
    iwfpm_plan_s* p;
    Solver* s;
    hipStream_t st;
    long long N;
    double2* col(int b, int j) const { return (double2*)s->buf[b].ptr + (size_t)j * N; }
};

#define CHECK_HIP(x)                                  \
    do {                                              \
        if ((x) != hipSuccess) return IWFPM_ERR_DEVICE; \
    } while (0)

static int sync(Ctx& c) {
    CHECK_HIP(hipStreamSynchronize(c.st));
    c.s->ring_since_sync = 0;
    return IWFPM_OK;
}

// C (p x q) = L^H R on the host, chunking both sides by kMaxCols
static int host_gram(Ctx& c, const std::vector<double2*>& L, const std::vector<double2*>& R, std::vector<cd>& C) {
    const int p = (int)L.size(), q = (int)R.size();
    C.assign((size_t)p * q, 0.0);
    // the reduction writes straight into the pinned (device-visible) host
    // mirror: no separate copy and its launch per Gram
    double2* h = c.s->hsmall;
    for (int i0 = 0; i0 < p; i0 += kMaxCols) {
        int pi = std::min(kMaxCols, p - i0);
        for (int j0 = 0; j0 < q; j0 += kMaxCols) {
            int qj = std::min(kMaxCols, q - j0);
            ColPtrs a{}, b{};
            for (int i = 0; i < pi; ++i) a.p[i] = L[i0 + i];
            for (int j = 0; j < qj; ++j) b.p[j] = R[j0 + j];
            CHECK_HIP(gram(a, pi, b, qj, c.N, (double2*)c.s->partial.ptr, c.s->max_blocks, h, c.st));
            if (int rc = sync(c)) return rc;
            for (int j = 0; j < qj; ++j)
                for (int i = 0; i < pi; ++i) {
                    double2 v = h[(size_t)j * pi + i];
                    C[(size_t)(i0 + i) + (size_t)(j0 + j) * p] = cd(v.x, v.y);
                }
        }
    }
    return IWFPM_OK;
}

// Y_j = beta Y_j + sum_i A_i C[(r0 + i) + j*ldc] for the q outputs
static int dev_lincomb(Ctx& c, const std::vector<double2*>& A, const std::vector<double2*>& Y, const std::vector<cd>& Cm,
                       int ldc, int r0, double beta) {
    const int p = (int)A.size(), q = (int)Y.size();
    if (q == 0) return IWFPM_OK;
    if (p == 0) {
        if (beta == 0.0)
            for (auto y : Y) CHECK_HIP(hipMemsetAsync(y, 0, c.N * sizeof(double2), c.st));
        return IWFPM_OK;
    }
    for (int j0 = 0; j0 < q; j0 += 48) {
        int qj = std::min(48, q - j0);
        for (int i0 = 0; i0 < p; i0 += kMaxCols) {  // later input chunks accumulate
            int pi = std::min(kMaxCols, p - i0);
            if (c.s->ring_since_sync >= kRingSlots - 1)
                if (int rc = sync(c)) return rc;
            int slot = c.s->ring_next;
            c.s->ring_next = (slot + 1) % kRingSlots;
            c.s->ring_since_sync++;
            double2* h = c.s->hring + (size_t)slot * kSlot;
            double2* dC = (double2*)c.s->dring.ptr + (size_t)slot * kSlot;
            for (int j = 0; j < qj; ++j)
                for (int i = 0; i < pi; ++i) {
                    cd v = Cm[(size_t)(r0 + i0 + i) + (size_t)(j0 + j) * ldc];
                    h[(size_t)j * pi + i] = make_double2(v.real(), v.imag());
                }
            CHECK_HIP(hipMemcpyAsync(dC, h, (size_t)pi * qj * sizeof(double2), hipMemcpyHostToDevice, c.st));
            ColPtrs a{}, y{};
            for (int i = 0; i < pi; ++i) a.p[i] = A[i0 + i];
            for (int j = 0; j < qj; ++j) y.p[j] = Y[j0 + j];
            CHECK_HIP(lincomb(a, pi, y, qj, dC, i0 == 0 ? beta : 1.0, c.N, c.st));
        }
    }
    return IWFPM_OK;
}

static std::vector<double2*> cols(Ctx& c, int b, int j0, int cnt) {
    std::vector<double2*> v(cnt);
    for (int j = 0; j < cnt; ++j) v[j] = c.col(b, j0 + j);
    return v;
}

template <class S>
static void hermitian_part(std::vector<S>& A, int n) {
    for (int j = 0; j < n; ++j) {
        A[j + (size_t)j * n] = real_(A[j + (size_t)j * n]);
        for (int i = 0; i < j; ++i) {
            S a = 0.5 * (A[i + (size_t)j * n] + conj_(A[j + (size_t)i * n]));
            A[i + (size_t)j * n] = a;
            A[j + (size_t)i * n] = conj_(a);
        }
    }
}

// Rayleigh-Ritz of X alone with X first made orthonormal again (the block
// updates keep it so only up to accumulated rounding): from the Gram
// G = X^H [X HX] (m x 2m), T = SVQB(X^H X) and the eigenvectors C of
// T^H (X^H H X) T; the update is X <- X (T C), HX <- HX (T C).  false if X
// has lost rank.
template <class S>
static bool rr_transform_t(const std::vector<S>& G, int m, std::vector<double>& theta, std::vector<S>& TC) {
    std::vector<S> Gxx(G.begin(), G.begin() + (size_t)m * m), T;
    if (svqb_t(Gxx, m, T, 1e-12) < m) return false;
    std::vector<S> A((size_t)m * m, 0.0), GT((size_t)m * m, 0.0);
    for (int j = 0; j < m; ++j)  // (X^H H X) T
        for (int i = 0; i < m; ++i) {
            S acc = 0.0;
            for (int k = 0; k < m; ++k) acc += G[(size_t)i + (size_t)(m + k) * m] * T[k + (size_t)j * m];
            GT[i + (size_t)j * m] = acc;
        }
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            S acc = 0.0;
            for (int k = 0; k < m; ++k) acc += conj_(T[k + (size_t)i * m]) * GT[k + (size_t)j * m];
            A[i + (size_t)j * m] = acc;
        }
    hermitian_part(A, m);
    std::vector<S> C;
    heev_t(A, m, theta, C);
    TC.assign((size_t)m * m, 0.0);
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            S acc = 0.0;
            for (int k = 0; k < m; ++k) acc += T[i + (size_t)k * m] * C[k + (size_t)j * m];
            TC[i + (size_t)j * m] = acc;
        }
    return true;
}

static bool rr_transform(const std::vector<cd>& G, int m, std::vector<double>& theta, std::vector<cd>& TC) {
    if (!exactly_real(G)) return rr_transform_t(G, m, theta, TC);
    std::vector<double> t;
    if (!rr_transform_t(real_parts(G), m, theta, t)) return false;
    TC = as_complex(t);
    return true;
}

// Rayleigh-Ritz in the coefficient space of the orthonormal basis
// S = [X W P] (ns columns, the first m are X): G = S^H [HW HP] (ns x (ns - m)),
// X^H H X = diag(theta).  Returns the Ritz values th (ascending, ns) and U =
// [C_x | Z T] (ns x 2m): the m lowest Ritz vectors, then the next P as the
// non-X part of the active Ritz vectors, orthogonalised against C_x and
// orthonormalised; the return value is the number of P columns.
template <class S>
static int rr_coefficients_t(const std::vector<S>& G, const std::vector<double>& theta, int m, int ns,
                             const std::vector<int>& act, std::vector<double>& th, std::vector<S>& U) {
    // small dense algebra: sums may be reassociated (vectorised); the result
    // is still the same for every run of one build
#pragma clang fp reassociate(on)
    const int ma = (int)act.size();
    std::vector<S> A((size_t)ns * ns, 0.0);
    const int nr = ns - m;
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < ns; ++i) {
            A[i + (size_t)(m + j) * ns] = G[i + (size_t)j * ns];
            if (i < m) A[(m + j) + (size_t)i * ns] = conj_(G[i + (size_t)j * ns]);
        }
    for (int j = 0; j < m; ++j) A[j + (size_t)j * ns] = theta[j];
    hermitian_part(A, ns);
    std::vector<S> Cfull;  // ns x m: the Ritz vectors of the m lowest values
    if (!heev_lowest_t(A, ns, m, th, Cfull)) heev_t(A, ns, th, Cfull);
    std::vector<S> Z((size_t)ns * m, 0.0);
    for (int a = 0; a < ma; ++a)
        for (int i = m; i < ns; ++i) Z[i + (size_t)a * ns] = Cfull[i + (size_t)act[a] * ns];
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<S> Gx((size_t)m * m, 0.0);  // C_x^H Z
        for (int j = 0; j < ma; ++j)
            for (int i = 0; i < m; ++i) {
                S acc = 0.0;
                for (int k = 0; k < ns; ++k) acc += conj_(Cfull[k + (size_t)i * ns]) * Z[k + (size_t)j * ns];
                Gx[i + (size_t)j * m] = acc;
            }
        for (int j = 0; j < ma; ++j)
            for (int k = 0; k < ns; ++k) {
                S acc = 0.0;
                for (int i = 0; i < m; ++i) acc += Cfull[k + (size_t)i * ns] * Gx[i + (size_t)j * m];
                Z[k + (size_t)j * ns] -= acc;
            }
    }
    int mpn = 0;
    U.assign((size_t)ns * (2 * m), 0.0);
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < ns; ++i) U[i + (size_t)j * ns] = Cfull[i + (size_t)j * ns];
    if (ns > m && ma > 0) {
        std::vector<S> Gz((size_t)ma * ma, 0.0), T;
        for (int j = 0; j < ma; ++j)
            for (int i = 0; i < ma; ++i) {
                S acc = 0.0;
                for (int k = 0; k < ns; ++k) acc += conj_(Z[k + (size_t)i * ns]) * Z[k + (size_t)j * ns];
                Gz[i + (size_t)j * ma] = acc;
            }
        double gmax = 0.0;
        for (int j = 0; j < ma; ++j) gmax = std::max(gmax, real_(Gz[j + (size_t)j * ma]));
        if (gmax > 1e-28) {
            mpn = svqb_t(Gz, ma, T, 1e-12);
            for (int j = 0; j < mpn; ++j)
                for (int i = 0; i < ns; ++i) {
                    S acc = 0.0;
                    for (int k = 0; k < ma; ++k) acc += Z[i + (size_t)k * ns] * T[k + (size_t)j * ma];
                    U[i + (size_t)(m + j) * ns] = acc;
                }
        }
    }
    return mpn;
}

static int rr_coefficients(const std::vector<cd>& G, const std::vector<double>& theta, int m, int ns,
                           const std::vector<int>& act, std::vector<double>& th, std::vector<cd>& U) {
    if (!exactly_real(G)) return rr_coefficients_t(G, theta, m, ns, act, th, U);
    std::vector<double> u;
    const int mpn = rr_coefficients_t(real_parts(G), theta, m, ns, act, th, u);
    U = as_complex(u);
    return mpn;
}

// Second projection and orthonormalisation of the new directions W (ma
// columns) against the orthonormal [X P] (nx columns), in coefficient space,
// after one explicit projection W <- W - [X P] ([X P]^H W).  Gall is the Gram
// [X P W]^H W ((nx + ma) x ma) of the projected W.  With G = [X P]^H W (now
// small: what the first projection left, including the effect of any loss of
// orthonormality in [X P] itself), the complement W - [X P] G has the Gram
// Gc = W^H W - G^H G, in which nothing cancels any more; SVQB of Gc gives T
// (dropping dependent directions) and the new block is [X P W] Cm,
// Cm = [-G T; T] ((nx + ma) x mw).  Together with the explicit first pass this
// is the classical project-twice scheme, with the second pass, the Gram of the
// result and its combination folded into one Gram and one combination.  (A
// single projection in coefficient space is not enough: it takes [X P] as
// exactly orthonormal, so any drift there passes into W and then into the
// next X and P, and accumulates.)  Returns false when the Gram is not finite
// or nothing is left (the caller then projects explicitly).
template <class S>
static bool ortho_coefficients_t(const std::vector<S>& Gall, int nx, int ma, std::vector<S>& Cm, int& mw) {
    // small dense algebra: sums may be reassociated (vectorised); the result
    // is still the same for every run of one build
#pragma clang fp reassociate(on)
    const int ld = nx + ma;
    std::vector<S> Gc((size_t)ma * ma);
    for (int j = 0; j < ma; ++j)
        for (int i = 0; i < ma; ++i) {
            S acc = Gall[(size_t)(nx + i) + (size_t)j * ld];
            for (int k = 0; k < nx; ++k) acc -= conj_(Gall[k + (size_t)i * ld]) * Gall[k + (size_t)j * ld];
            Gc[i + (size_t)j * ma] = acc;
        }
    for (int j = 0; j < ma; ++j)
        if (!std::isfinite(real_(Gc[j + (size_t)j * ma])) || !(real_(Gc[j + (size_t)j * ma]) > 0.0)) return false;
    hermitian_part(Gc, ma);
    std::vector<S> T;
    mw = svqb_t(Gc, ma, T, 1e-10);
    if (mw < 1) return false;
    Cm.assign((size_t)ld * mw, 0.0);
    for (int c = 0; c < mw; ++c) {
        for (int i = 0; i < ma; ++i) Cm[(size_t)(nx + i) + (size_t)c * ld] = T[i + (size_t)c * ma];
        for (int k = 0; k < nx; ++k) {
            S acc = 0.0;
            for (int i = 0; i < ma; ++i) acc += Gall[k + (size_t)i * ld] * T[i + (size_t)c * ma];
            Cm[k + (size_t)c * ld] = -acc;
        }
    }
    return true;
}

static bool ortho_coefficients(const std::vector<cd>& Gall, int nx, int ma, std::vector<cd>& Cm, int& mw) {
    if (!exactly_real(Gall)) return ortho_coefficients_t(Gall, nx, ma, Cm, mw);
    std::vector<double> c;
    if (!ortho_coefficients_t(real_parts(Gall), nx, ma, c, mw)) return false;
    Cm = as_complex(c);
    return true;
}

// -G (the [X P] rows of a Gram [X P W]^H W, negated): the coefficients of one
// explicit projection W <- W - [X P] G
static std::vector<cd> neg_projection(const std::vector<cd>& Gall, int nx, int ma) {
    std::vector<cd> G((size_t)nx * ma);
    for (int j = 0; j < ma; ++j)
        for (int k = 0; k < nx; ++k) G[k + (size_t)j * nx] = -Gall[k + (size_t)j * (nx + ma)];
    return G;
}

// IWFPM_ORTHO=explicit: always project explicitly twice and apply SVQB to the
// result (the route taken when the coefficient-space second pass fails)
static bool force_explicit_ortho() {
    const char* e = std::getenv("IWFPM_ORTHO");
    return e && std::strcmp(e, "explicit") == 0;
}

// ---------------------------------------------------------------------------
// Real-symmetric LOBPCG.  When every Vhat_m is real (Hermiticity then makes
// V even), H~ is a real symmetric matrix and its eigenvectors can be taken
// real: the solver then works on real trial vectors stored two per complex
// column (real part, imaginary part).  The apply maps such a pair to its image
// pair (H~ is real), the preconditioners act on both halves alike, and the
// block algebra uses the pair kernels (four real Gram accumulators per tile,
// 2 x 2 real coefficient blocks).  Small matrices are kept as complex arrays
// with zero imaginary parts: the host solvers keep such inputs exactly real.
// ---------------------------------------------------------------------------

// real vector v of a block buffer: part v & 1 of column v >> 1
struct RVec {
    double2* col;
    int part;
};

static std::vector<RVec> rvecs(Ctx& c, int b, int v0, int cnt) {
    std::vector<RVec> r(cnt);
    for (int k = 0; k < cnt; ++k) r[k] = {c.col(b, (v0 + k) >> 1), (v0 + k) & 1};
    return r;
}

// distinct columns of a list of real vectors (first-seen order) and, per
// vector, 2 * (its column's position) + part
struct PairCols {
    std::vector<double2*> cols;
    std::vector<int> at;
};

static PairCols pair_cols(const std::vector<RVec>& v) {
    PairCols pc;
    for (const RVec& x : v) {
        int ci = -1;
        for (size_t j = 0; j < pc.cols.size(); ++j)
            if (pc.cols[j] == x.col) {
                ci = (int)j;
                break;
            }
        if (ci < 0) {
            ci = (int)pc.cols.size();
            pc.cols.push_back(x.col);
        }
        pc.at.push_back(2 * ci + x.part);
    }
    return pc;
}

// G (|L| x |R|, real, zero imaginary parts) = L^T R over real vectors
static int host_gram_real(Ctx& c, const std::vector<RVec>& L, const std::vector<RVec>& R, std::vector<cd>& G) {
    const PairCols Lp = pair_cols(L), Rp = pair_cols(R);
    const int P = (int)Lp.cols.size(), Q = (int)Rp.cols.size();
    const size_t ldf = 2 * (size_t)P;
    std::vector<double> Gf(ldf * 2 * (size_t)Q, 0.0);
    double* h = (double*)c.s->hsmall;  // written by the reduction directly (pinned, device-visible)
    constexpr int kc = kMaxCols / 2;
    for (int i0 = 0; i0 < P; i0 += kc) {
        const int pi = std::min(kc, P - i0);
        for (int j0 = 0; j0 < Q; j0 += kc) {
            const int qj = std::min(kc, Q - j0);
            ColPtrs a{}, b{};
            for (int i = 0; i < pi; ++i) a.p[i] = Lp.cols[i0 + i];
            for (int j = 0; j < qj; ++j) b.p[j] = Rp.cols[j0 + j];
            CHECK_HIP(gram_pairs(a, pi, b, qj, c.N, (double2*)c.s->partial.ptr, c.s->max_blocks, h, c.st));
            if (int rc = sync(c)) return rc;
            for (int s2 = 0; s2 < 2 * qj; ++s2)
                for (int r2 = 0; r2 < 2 * pi; ++r2)
                    Gf[(size_t)(2 * i0 + r2) + (size_t)(2 * j0 + s2) * ldf] = h[(size_t)r2 + (size_t)s2 * 2 * pi];
        }
    }
    const int nl = (int)L.size(), nr = (int)R.size();
    G.assign((size_t)nl * nr, 0.0);
    for (int l = 0; l < nr; ++l)
        for (int k = 0; k < nl; ++k) G[k + (size_t)l * nl] = Gf[(size_t)Lp.at[k] + (size_t)Rp.at[l] * ldf];
    return IWFPM_OK;
}

// Y_l = beta Y_l + sum_k A_k Re C[(r0 + k) + l * ldc] over real vectors; the
// outputs fill whole columns from their first half (a half with no output
// vector receives beta times itself plus zero)
static int dev_lincomb_real(Ctx& c, const std::vector<RVec>& A, const std::vector<RVec>& Y, const std::vector<cd>& Cm,
                            int ldc, int r0, double beta) {
    if (Y.empty()) return IWFPM_OK;
    const PairCols Ap = pair_cols(A), Yp = pair_cols(Y);
    const int P = (int)Ap.cols.size(), Q = (int)Yp.cols.size();
    if (Q > 32) return IWFPM_ERR_ARG;
    if (P == 0) {
        if (beta == 0.0)
            for (auto y : Yp.cols) CHECK_HIP(hipMemsetAsync(y, 0, c.N * sizeof(double2), c.st));
        return IWFPM_OK;
    }
    constexpr int kc = kMaxCols / 2;  // input columns per call
    for (int i0 = 0; i0 < P; i0 += kc) {
        const int pi = std::min(kc, P - i0);
        if (c.s->ring_since_sync >= kRingSlots - 1)
            if (int rc = sync(c)) return rc;
        const int slot = c.s->ring_next;
        c.s->ring_next = (slot + 1) % kRingSlots;
        c.s->ring_since_sync++;
        double* h = (double*)(c.s->hring + (size_t)slot * kSlot);
        double* dC = (double*)((double2*)c.s->dring.ptr + (size_t)slot * kSlot);
        const size_t ld = 2 * (size_t)pi;
        std::fill(h, h + ld * 2 * (size_t)Q, 0.0);
        for (size_t k = 0; k < A.size(); ++k) {
            const int row = Ap.at[k] - 2 * i0;
            if (row < 0 || row >= (int)ld) continue;
            for (size_t l = 0; l < Y.size(); ++l)
                h[(size_t)row + (size_t)Yp.at[l] * ld] = Cm[(size_t)(r0 + k) + l * (size_t)ldc].real();
        }
        CHECK_HIP(hipMemcpyAsync(dC, h, ld * 2 * (size_t)Q * sizeof(double), hipMemcpyHostToDevice, c.st));
        ColPtrs a{}, y{};
        for (int i = 0; i < pi; ++i) a.p[i] = Ap.cols[i0 + i];
        for (int j = 0; j < Q; ++j) y.p[j] = Yp.cols[j];
        CHECK_HIP(lincomb_pairs(a, pi, y, Q, dC, i0 == 0 ? beta : 1.0, c.N, c.st));
    }
    return IWFPM_OK;
}

static ColPtrs colptrs(const std::vector<RVec>& v, unsigned long long* parts) {
    ColPtrs cp{};
    *parts = 0;
    for (size_t k = 0; k < v.size(); ++k) {
        cp.p[k] = v[k].col;
        if (v[k].part) *parts |= 1ull << k;
    }
    return cp;
}

// Rayleigh-Ritz on X alone: X <- X C, HX <- HX C (real)
// every potential coefficient real: H~ is real symmetric
static bool real_symmetric(const iwfpm_plan_s* p) {
    for (double v : p->vim)
        if (v != 0.0) return false;
    return true;
}


// ---------------------------------------------------------------------------
// lock-step block LOBPCG for a batch of plans (e.g. a sweep of couplings):
// every tall operation of one phase runs for all live instances in a single
// launch (job tables), the applies go through one persistent batched launch
// (replayed from a hipGraph), and the per-instance small problems run on
// host threads.
// ---------------------------------------------------------------------------

template <class F>
static void parallel_for(int n, F&& f) {
    int nt = std::min<int>(n, std::min(16u, std::max(1u, std::thread::hardware_concurrency())));
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&]() {
            for (int i; (i = next.fetch_add(1)) < n;) f(i);
        });
    for (auto& x : th) x.join();
}

struct BatchOps {
    hipStream_t st = nullptr;
    DeviceBuf d_jobs, d_coef, d_partial, d_out;
    unsigned char* h_jobs = nullptr;
    double2* h_coef = nullptr;
    double2* h_out = nullptr;
    size_t jobs_cap = 0, coef_cap = 0, partial_cap = 0, out_cap = 0;
    hipEvent_t staged = nullptr;
    ~BatchOps() {
        if (staged) {
            (void)hipEventSynchronize(staged);
            (void)hipEventDestroy(staged);
        }
        dev_free(d_jobs);
        dev_free(d_coef);
        dev_free(d_partial);
        dev_free(d_out);
        if (h_jobs) (void)hipHostFree(h_jobs);
        if (h_coef) (void)hipHostFree(h_coef);
        if (h_out) (void)hipHostFree(h_out);
    }
    int reserve_host(void** h, size_t& cap, size_t need) {
        if (need <= cap) return IWFPM_OK;
        if (staged) (void)hipEventSynchronize(staged);
        if (*h) (void)hipHostFree(*h);
        *h = nullptr;
        cap = 0;
        if (hipHostMalloc(h, need) != hipSuccess) return IWFPM_ERR_ALLOC;
        cap = need;
        return IWFPM_OK;
    }
    int reserve_dev(DeviceBuf& b, size_t need) {
        if (b.bytes >= need) return IWFPM_OK;
        if (hipStreamSynchronize(st) != hipSuccess) return IWFPM_ERR_DEVICE;
        return dev_alloc(b, need);
    }
    // the host staging buffers may be rewritten once the last upload is done
    int wait_staged() { return staged && hipEventSynchronize(staged) != hipSuccess ? IWFPM_ERR_DEVICE : IWFPM_OK; }
};

struct GramReq {
    std::vector<double2*> L, R;
    long long N;
};

// C_k = L_k^H R_k for every request, one launch (two with the reduction)
static int batch_gram(BatchOps& bo, const std::vector<GramReq>& reqs, std::vector<std::vector<cd>>& out) {
    struct Sub {
        int req, i0, j0;
    };
    std::vector<GramJob> jobs;
    std::vector<Sub> subs;
    long long part = 0;
    int blocks = 0, outs = 0, maxp = 1, maxq = 1;
    for (int r = 0; r < (int)reqs.size(); ++r) {
        const int p = (int)reqs[r].L.size(), q = (int)reqs[r].R.size();
        for (int i0 = 0; i0 < p; i0 += kMaxCols)
            for (int j0 = 0; j0 < q; j0 += kMaxCols) {
                GramJob jb{};
                jb.p = std::min(kMaxCols, p - i0);
                jb.q = std::min(kMaxCols, q - j0);
                for (int i = 0; i < jb.p; ++i) jb.L.p[i] = reqs[r].L[i0 + i];
                for (int j = 0; j < jb.q; ++j) jb.R.p[j] = reqs[r].R[j0 + j];
                jb.N = reqs[r].N;
                jb.nb = gram_job_blocks(jb.p, jb.N, 256, &jb.groups_per_block);
                maxp = std::max(maxp, jb.p);
                maxq = std::max(maxq, jb.q);
                jb.start = blocks;
                jb.out_start = outs;
                jb.part_off = part;
                blocks += jb.nb;
                outs += jb.p * jb.q;
                part += (long long)jb.nb * jb.p * jb.q;
                jobs.push_back(jb);
                subs.push_back({r, i0, j0});
            }
    }
    out.assign(reqs.size(), {});
    for (size_t r = 0; r < reqs.size(); ++r) out[r].assign(reqs[r].L.size() * reqs[r].R.size(), 0.0);
    if (jobs.empty()) return IWFPM_OK;
    int rc;
    if ((rc = bo.wait_staged())) return rc;
    if ((rc = bo.reserve_host((void**)&bo.h_jobs, bo.jobs_cap, jobs.size() * sizeof(GramJob)))) return rc;
    if ((rc = bo.reserve_host((void**)&bo.h_out, bo.out_cap, (size_t)outs * sizeof(double2)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_jobs, jobs.size() * sizeof(GramJob)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_partial, (size_t)part * sizeof(double2)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_out, (size_t)outs * sizeof(double2)))) return rc;
    std::memcpy(bo.h_jobs, jobs.data(), jobs.size() * sizeof(GramJob));
    CHECK_HIP(hipMemcpyAsync(bo.d_jobs.ptr, bo.h_jobs, jobs.size() * sizeof(GramJob), hipMemcpyHostToDevice, bo.st));
    CHECK_HIP(gram_batched((const GramJob*)bo.d_jobs.ptr, (int)jobs.size(), blocks, outs, maxp, maxq,
                           (double2*)bo.d_partial.ptr, (double2*)bo.d_out.ptr, bo.st));
    CHECK_HIP(hipMemcpyAsync(bo.h_out, bo.d_out.ptr, (size_t)outs * sizeof(double2), hipMemcpyDeviceToHost, bo.st));
    CHECK_HIP(hipStreamSynchronize(bo.st));
    for (size_t k = 0; k < jobs.size(); ++k) {
        const GramJob& jb = jobs[k];
        const Sub& sb = subs[k];
        const int p = (int)reqs[sb.req].L.size();
        for (int j = 0; j < jb.q; ++j)
            for (int i = 0; i < jb.p; ++i) {
                double2 v = bo.h_out[jb.out_start + (size_t)j * jb.p + i];
                out[sb.req][(size_t)(sb.i0 + i) + (size_t)(sb.j0 + j) * p] = cd(v.x, v.y);
            }
    }
    return IWFPM_OK;
}

struct LinReq {
    std::vector<double2*> A, Y;
    const std::vector<cd>* C;
    int ldc, r0;
    double beta;
    long long N;
};

// Y_k = beta Y_k + A_k C_k for every request, one launch (inputs <= 64)
static int batch_lincomb(BatchOps& bo, const std::vector<LinReq>& reqs) {
    std::vector<LinJob> jobs;
    std::vector<size_t> coef_off;
    size_t coefs = 0;
    int blocks = 0, maxq = 1;
    for (const LinReq& r : reqs) {
        const int p = (int)r.A.size(), q = (int)r.Y.size();
        if (q == 0) continue;
        if (p > kMaxCols) return IWFPM_ERR_ARG;
        for (int j0 = 0; j0 < q; j0 += 48) {
            LinJob jb{};
            jb.p = p;
            jb.q = std::min(48, q - j0);
            for (int i = 0; i < p; ++i) jb.A.p[i] = r.A[i];
            for (int j = 0; j < jb.q; ++j) jb.Y.p[j] = r.Y[j0 + j];
            jb.beta = r.beta;
            jb.N = r.N;
            jb.nb = (int)std::min<long long>(1024, std::max<long long>(1, (r.N + 127) / 128));
            jb.start = blocks;
            blocks += jb.nb;
            maxq = std::max(maxq, jb.q);
            coef_off.push_back(coefs);
            coefs += (size_t)p * jb.q;
            jobs.push_back(jb);
        }
    }
    if (jobs.empty()) return IWFPM_OK;
    int rc;
    if ((rc = bo.wait_staged())) return rc;
    if ((rc = bo.reserve_host((void**)&bo.h_jobs, bo.jobs_cap, jobs.size() * sizeof(LinJob)))) return rc;
    if ((rc = bo.reserve_host((void**)&bo.h_coef, bo.coef_cap, std::max<size_t>(1, coefs) * sizeof(double2)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_jobs, jobs.size() * sizeof(LinJob)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_coef, std::max<size_t>(1, coefs) * sizeof(double2)))) return rc;
    size_t k = 0;
    for (const LinReq& r : reqs) {
        const int p = (int)r.A.size(), q = (int)r.Y.size();
        if (q == 0) continue;
        for (int j0 = 0; j0 < q; j0 += 48, ++k) {
            LinJob& jb = jobs[k];
            double2* h = bo.h_coef + coef_off[k];
            for (int j = 0; j < jb.q; ++j)
                for (int i = 0; i < p; ++i) {
                    cd v = (*r.C)[(size_t)(r.r0 + i) + (size_t)(j0 + j) * r.ldc];
                    h[(size_t)j * p + i] = make_double2(v.real(), v.imag());
                }
            jb.C = (const double2*)bo.d_coef.ptr + coef_off[k];
        }
    }
    std::memcpy(bo.h_jobs, jobs.data(), jobs.size() * sizeof(LinJob));
    CHECK_HIP(hipMemcpyAsync(bo.d_coef.ptr, bo.h_coef, coefs * sizeof(double2), hipMemcpyHostToDevice, bo.st));
    CHECK_HIP(hipMemcpyAsync(bo.d_jobs.ptr, bo.h_jobs, jobs.size() * sizeof(LinJob), hipMemcpyHostToDevice, bo.st));
    CHECK_HIP(hipEventRecord(bo.staged, bo.st));
    CHECK_HIP(lincomb_batched((const LinJob*)bo.d_jobs.ptr, (int)jobs.size(), blocks, maxq, bo.st));
    return IWFPM_OK;
}

// batched Grams and combinations over real trial vectors (two per column)

struct GramReqR {
    std::vector<RVec> L, R;
    long long N;
};

// G_k (|L| x |R| real, zero imaginary parts) for every request, one launch (two with the reduction)
static int batch_gram_real(BatchOps& bo, const std::vector<GramReqR>& reqs, std::vector<std::vector<cd>>& out) {
    std::vector<GramJob> jobs;
    std::vector<PairCols> Lp, Rp;
    long long part = 0;
    int blocks = 0, outs = 0, maxp = 1, maxq = 1;
    for (const GramReqR& r : reqs) {
        Lp.push_back(pair_cols(r.L));
        Rp.push_back(pair_cols(r.R));
        GramJob jb{};
        jb.p = (int)Lp.back().cols.size();
        jb.q = (int)Rp.back().cols.size();
        if (jb.p > kMaxCols / 2 || jb.q > kMaxCols / 2) return IWFPM_ERR_ARG;
        for (int i = 0; i < jb.p; ++i) jb.L.p[i] = Lp.back().cols[i];
        for (int j = 0; j < jb.q; ++j) jb.R.p[j] = Rp.back().cols[j];
        jb.N = r.N;
        jb.width = 2;
        jb.nb = gram_job_blocks(jb.p, jb.N, 256, &jb.groups_per_block);
        maxp = std::max(maxp, jb.p);
        maxq = std::max(maxq, jb.q);
        jb.start = blocks;
        jb.out_start = outs;
        jb.part_off = part;
        blocks += jb.nb;
        outs += 2 * jb.p * jb.q;
        part += (long long)jb.nb * 2 * jb.p * jb.q;
        jobs.push_back(jb);
    }
    out.assign(reqs.size(), {});
    if (jobs.empty()) return IWFPM_OK;
    int rc;
    if ((rc = bo.wait_staged())) return rc;
    if ((rc = bo.reserve_host((void**)&bo.h_jobs, bo.jobs_cap, jobs.size() * sizeof(GramJob)))) return rc;
    if ((rc = bo.reserve_host((void**)&bo.h_out, bo.out_cap, (size_t)outs * sizeof(double2)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_jobs, jobs.size() * sizeof(GramJob)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_partial, (size_t)part * sizeof(double2)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_out, (size_t)outs * sizeof(double2)))) return rc;
    std::memcpy(bo.h_jobs, jobs.data(), jobs.size() * sizeof(GramJob));
    CHECK_HIP(hipMemcpyAsync(bo.d_jobs.ptr, bo.h_jobs, jobs.size() * sizeof(GramJob), hipMemcpyHostToDevice, bo.st));
    CHECK_HIP(gram_batched_pairs((const GramJob*)bo.d_jobs.ptr, (int)jobs.size(), blocks, outs, maxp, maxq,
                                 (double2*)bo.d_partial.ptr, (double2*)bo.d_out.ptr, bo.st));
    CHECK_HIP(hipMemcpyAsync(bo.h_out, bo.d_out.ptr, (size_t)outs * sizeof(double2), hipMemcpyDeviceToHost, bo.st));
    CHECK_HIP(hipStreamSynchronize(bo.st));
    for (size_t k = 0; k < jobs.size(); ++k) {
        const double* g = (const double*)(bo.h_out + jobs[k].out_start);  // 2p x 2q real, column-major
        const size_t ld = 2 * (size_t)jobs[k].p;
        const int nl = (int)reqs[k].L.size(), nr = (int)reqs[k].R.size();
        out[k].assign((size_t)nl * nr, 0.0);
        for (int l = 0; l < nr; ++l)
            for (int i = 0; i < nl; ++i)
                out[k][i + (size_t)l * nl] = g[(size_t)Lp[k].at[i] + (size_t)Rp[k].at[l] * ld];
    }
    return IWFPM_OK;
}

struct LinReqR {
    std::vector<RVec> A, Y;  // Y: the first vectors of one or more buffers, filling columns from the first half
    const std::vector<cd>* C;
    int ldc, r0;
    double beta;
    long long N;
};

// Y_k = beta Y_k + A_k Re C_k for every request, one launch
static int batch_lincomb_real(BatchOps& bo, const std::vector<LinReqR>& reqs) {
    std::vector<LinJob> jobs;
    std::vector<PairCols> Ap, Yp;
    std::vector<size_t> coef_off;
    size_t coefs = 0;  // in double2 units
    int blocks = 0, maxq = 1;
    for (const LinReqR& r : reqs) {
        if (r.Y.empty()) continue;
        Ap.push_back(pair_cols(r.A));
        Yp.push_back(pair_cols(r.Y));
        LinJob jb{};
        jb.p = (int)Ap.back().cols.size();
        jb.q = (int)Yp.back().cols.size();
        if (jb.p > kMaxCols || jb.q > 32) return IWFPM_ERR_ARG;
        // the kernel stages the 2p x q coefficient pairs in an LDS array of
        // kLinPairsLds double2 entries
        if (2 * jb.p * jb.q > kLinPairsLds) return IWFPM_ERR_ARG;
        for (int i = 0; i < jb.p; ++i) jb.A.p[i] = Ap.back().cols[i];
        for (int j = 0; j < jb.q; ++j) jb.Y.p[j] = Yp.back().cols[j];
        jb.beta = r.beta;
        jb.N = r.N;
        jb.nb = (int)std::min<long long>(1024, std::max<long long>(1, (r.N + 127) / 128));
        jb.start = blocks;
        blocks += jb.nb;
        maxq = std::max(maxq, jb.q);
        coef_off.push_back(coefs);
        coefs += (size_t)2 * jb.p * jb.q;
        jobs.push_back(jb);
    }
    if (jobs.empty()) return IWFPM_OK;
    int rc;
    if ((rc = bo.wait_staged())) return rc;
    if ((rc = bo.reserve_host((void**)&bo.h_jobs, bo.jobs_cap, jobs.size() * sizeof(LinJob)))) return rc;
    if ((rc = bo.reserve_host((void**)&bo.h_coef, bo.coef_cap, std::max<size_t>(1, coefs) * sizeof(double2)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_jobs, jobs.size() * sizeof(LinJob)))) return rc;
    if ((rc = bo.reserve_dev(bo.d_coef, std::max<size_t>(1, coefs) * sizeof(double2)))) return rc;
    size_t k = 0;
    for (const LinReqR& r : reqs) {
        if (r.Y.empty()) continue;
        LinJob& jb = jobs[k];
        double* h = (double*)(bo.h_coef + coef_off[k]);
        const size_t ld = 2 * (size_t)jb.p;
        std::fill(h, h + ld * 2 * (size_t)jb.q, 0.0);
        for (size_t a = 0; a < r.A.size(); ++a)
            for (size_t l = 0; l < r.Y.size(); ++l)
                h[(size_t)Ap[k].at[a] + (size_t)Yp[k].at[l] * ld] =
                    (*r.C)[(size_t)(r.r0 + a) + l * (size_t)r.ldc].real();
        jb.C = (const double2*)bo.d_coef.ptr + coef_off[k];
        ++k;
    }
    std::memcpy(bo.h_jobs, jobs.data(), jobs.size() * sizeof(LinJob));
    CHECK_HIP(hipMemcpyAsync(bo.d_coef.ptr, bo.h_coef, coefs * sizeof(double2), hipMemcpyHostToDevice, bo.st));
    CHECK_HIP(hipMemcpyAsync(bo.d_jobs.ptr, bo.h_jobs, jobs.size() * sizeof(LinJob), hipMemcpyHostToDevice, bo.st));
    CHECK_HIP(hipEventRecord(bo.staged, bo.st));
    CHECK_HIP(lincomb_pairs_batched((const LinJob*)bo.d_jobs.ptr, (int)jobs.size(), blocks, maxq, bo.st));
    return IWFPM_OK;
}


// ---------------------------------------------------------------------------
// Block LOBPCG for the lowest eigenpairs of H~ (Knyazev's method with soft
// locking; the reading of the paper's Alg. 2 is the block method for the
// smallest eigenvalues of the Hermitian matrix): one iteration body for a
// single solve (B = 1) and for B plans in lock step, over both ways of holding
// the trial vectors.
//   CplxRoute: one trial vector per complex column.
//   RealRoute: every potential coefficient real, so H~ is real symmetric and
//              its eigenvectors can be taken real: real trial vectors, two per
//              complex column (real part, imaginary part); the apply maps a
//              pair to its image pair, the preconditioners act on both halves
//              alike, the block algebra runs on the pair kernels (2 x 2 real
//              coefficient blocks), and the small matrices are complex arrays
//              with zero imaginary parts, which the host solvers keep real.
// Every tall operation of a phase runs for all live instances together: a
// single solve through the one-plan kernels (Grams reduced on the device and
// read back, combinations with coefficients staged through a ring of slots),
// a batch through one launch over a job table per phase; the applies of a
// batch go through its persistent, graph-replayed batched launch; the small
// dense problems run on host threads, one per instance.
// ---------------------------------------------------------------------------

struct CplxRoute {
    using V = double2*;
    static constexpr bool real = false;
    static std::vector<V> vecs(Ctx& c, int b, int v0, int cnt) { return cols(c, b, v0, cnt); }
    static int columns(int nv) { return nv; }
};
struct RealRoute {
    using V = RVec;
    static constexpr bool real = true;
    static std::vector<V> vecs(Ctx& c, int b, int v0, int cnt) { return rvecs(c, b, v0, cnt); }
    static int columns(int nv) { return (nv + 1) / 2; }
};

// one solve of the batch
struct BInst {
    iwfpm_plan_s* p = nullptr;
    Solver* s = nullptr;
    Ctx c{};
    int prec = 0;
    bool can64 = false;
    bool done = false;
    bool cleaned = false;  // X re-orthonormalised since its pairs converged
    int status = IWFPM_OK;
    std::vector<double> theta, eta;
    int mp = 0, it = 0, polished = 0, reortho = 0;
    long long matvecs = 0;
    double best_eta = 1e300, floor32 = 0.0, hnorm = 0.0;
    int best_it = 0;
    LearnedPrecond* lp = nullptr;  // learned preconditioner while it is in use
    int fallback = 0;
    // per-iteration
    std::vector<int> act;
    int ma = 0, mq = 0, mw = 0, ns = 0;
    bool lp_used = false;
    std::vector<cd> T, U;
    std::vector<double> th;
    int mpn = 0;
};

template <class Rt>
struct GramQ {
    Ctx* c;
    std::vector<typename Rt::V> L, R;
};
template <class Rt>
struct LinQ {
    Ctx* c;
    std::vector<typename Rt::V> A, Y;
    const std::vector<cd>* C;
    int ldc;
    double beta;
};

// the tall operations of one phase, for a single solve or a batch
struct Tall {
    BatchOps bo;
    bool single = true;
};

template <class Rt>
static int tall_grams(Tall& t, const std::vector<GramQ<Rt>>& q, std::vector<std::vector<cd>>& out) {
    if (t.single) {
        out.assign(q.size(), {});
        for (size_t k = 0; k < q.size(); ++k) {
            int rc;
            if constexpr (Rt::real) rc = host_gram_real(*q[k].c, q[k].L, q[k].R, out[k]);
            else rc = host_gram(*q[k].c, q[k].L, q[k].R, out[k]);
            if (rc) return rc;
        }
        return IWFPM_OK;
    }
    if constexpr (Rt::real) {
        std::vector<GramReqR> r;
        for (const auto& x : q) r.push_back({x.L, x.R, x.c->N});
        return batch_gram_real(t.bo, r, out);
    } else {
        std::vector<GramReq> r;
        for (const auto& x : q) r.push_back({x.L, x.R, x.c->N});
        return batch_gram(t.bo, r, out);
    }
}

template <class Rt>
static int tall_lincombs(Tall& t, const std::vector<LinQ<Rt>>& q) {
    if (t.single) {
        for (const auto& x : q) {
            int rc;
            if constexpr (Rt::real) rc = dev_lincomb_real(*x.c, x.A, x.Y, *x.C, x.ldc, 0, x.beta);
            else rc = dev_lincomb(*x.c, x.A, x.Y, *x.C, x.ldc, 0, x.beta);
            if (rc) return rc;
        }
        return IWFPM_OK;
    }
    if constexpr (Rt::real) {
        std::vector<LinReqR> r;
        for (const auto& x : q) r.push_back({x.A, x.Y, x.C, x.ldc, 0, x.beta, x.c->N});
        return batch_lincomb_real(t.bo, r);
    } else {
        std::vector<LinReq> r;
        for (const auto& x : q) r.push_back({x.A, x.Y, x.C, x.ldc, 0, x.beta, x.c->N});
        return batch_lincomb(t.bo, r);
    }
}

// R = HX - X theta and eta_j = |r_j| / ((|H|_est + |theta_j|) |x_j|) (x_j
// unit) for every live instance; a non-finite value ends that instance
template <class Rt>
static int tall_residuals(Tall& t, std::vector<BInst>& in, const std::vector<int>& live, int m) {
    const int mc = Rt::columns(m);
    const int per = Rt::real ? 2 * mc : m;  // norms per instance
    std::vector<double> nrm((size_t)live.size() * per, 0.0);
    if (t.single) {
        for (size_t k = 0; k < live.size(); ++k) {
            BInst& b = in[live[k]];
            ColPtrs hx{}, x{}, r{};
            Reals th{};
            for (int j = 0; j < mc; ++j) {
                hx.p[j] = b.c.col(B_HX, j);
                x.p[j] = b.c.col(B_X, j);
                r.p[j] = b.c.col(B_T1, j);
            }
            for (int v = 0; v < per; ++v) th.v[v] = v < m ? b.theta[v] : 0.0;
            // the norms land in the pinned host mirror directly
            double* h = (double*)(b.s->hsmall + 96 * 96);
            if constexpr (Rt::real)
                CHECK_HIP(residual_norm_pairs(hx, x, r, th, mc, b.c.N, (double*)b.s->partial.ptr, b.s->max_blocks, h,
                                              b.c.st));
            else
                CHECK_HIP(residual_norm(hx, x, r, th, m, b.c.N, (double*)b.s->partial.ptr, b.s->max_blocks, h,
                                        b.c.st));
            if (int rc = sync(b.c)) return rc;
            std::copy(h, h + per, nrm.begin() + (size_t)k * per);
        }
    } else {
        BatchOps& bo = t.bo;
        std::vector<ResJob> jobs;
        int blocks = 0, outs = 0;
        long long part = 0;
        for (int i : live) {
            BInst& b = in[i];
            ResJob jb{};
            for (int j = 0; j < mc; ++j) {
                jb.HX.p[j] = b.c.col(B_HX, j);
                jb.X.p[j] = b.c.col(B_X, j);
                jb.R.p[j] = b.c.col(B_T1, j);
            }
            for (int v = 0; v < per; ++v) jb.theta.v[v] = v < m ? b.theta[v] : 0.0;
            jb.m = mc;
            if (Rt::real) jb.width = 2;
            jb.N = b.c.N;
            jb.nb = (int)std::min<long long>(256, std::max<long long>(1, (jb.N + 1023) / 1024));
            jb.rows_per_block = (jb.N + jb.nb - 1) / jb.nb;
            jb.start = blocks;
            jb.out_start = outs;
            jb.part_off = part;
            blocks += jb.nb;
            outs += per;
            part += (long long)jb.nb * per;
            jobs.push_back(jb);
        }
        int rc;
        if ((rc = bo.wait_staged())) return rc;
        if ((rc = bo.reserve_host((void**)&bo.h_jobs, bo.jobs_cap, jobs.size() * sizeof(ResJob)))) return rc;
        if ((rc = bo.reserve_host((void**)&bo.h_out, bo.out_cap, (size_t)outs * sizeof(double2)))) return rc;
        if ((rc = bo.reserve_dev(bo.d_jobs, jobs.size() * sizeof(ResJob)))) return rc;
        if ((rc = bo.reserve_dev(bo.d_partial, (size_t)part * sizeof(double2)))) return rc;
        if ((rc = bo.reserve_dev(bo.d_out, (size_t)outs * sizeof(double2)))) return rc;
        std::memcpy(bo.h_jobs, jobs.data(), jobs.size() * sizeof(ResJob));
        CHECK_HIP(hipMemcpyAsync(bo.d_jobs.ptr, bo.h_jobs, jobs.size() * sizeof(ResJob), hipMemcpyHostToDevice, bo.st));
        if constexpr (Rt::real)
            CHECK_HIP(residual_norm_pairs_batched((const ResJob*)bo.d_jobs.ptr, (int)jobs.size(), blocks, outs,
                                                  (double*)bo.d_partial.ptr, (double*)bo.d_out.ptr, bo.st));
        else
            CHECK_HIP(residual_norm_batched((const ResJob*)bo.d_jobs.ptr, (int)jobs.size(), blocks, outs,
                                            (double*)bo.d_partial.ptr, (double*)bo.d_out.ptr, bo.st));
        CHECK_HIP(hipMemcpyAsync(bo.h_out, bo.d_out.ptr, outs * sizeof(double), hipMemcpyDeviceToHost, bo.st));
        CHECK_HIP(hipStreamSynchronize(bo.st));
        const double* h = (const double*)bo.h_out;
        std::copy(h, h + outs, nrm.begin());
    }
    for (size_t k = 0; k < live.size(); ++k) {
        BInst& b = in[live[k]];
        for (int j = 0; j < m; ++j) {
            b.eta[j] = std::sqrt(std::max(0.0, nrm[k * per + j])) / (b.hnorm + std::fabs(b.theta[j]));
            if (!std::isfinite(b.eta[j]) || !std::isfinite(b.theta[j])) {
                b.done = true;
                b.status = IWFPM_ERR_NUMERIC;
            }
        }
    }
    return IWFPM_OK;
}

// W = M R_A of one instance with the plain preconditioner (one-plan kernels)
template <class Rt>
static int plain_precondition(BInst& b) {
    if constexpr (Rt::real) {
        std::vector<RVec> Ract(b.ma);
        for (int a = 0; a < b.ma; ++a) Ract[a] = {b.c.col(B_T1, b.act[a] >> 1), b.act[a] & 1};
        unsigned long long parts = 0;
        const ColPtrs src = colptrs(Ract, &parts);
        ColPtrs w{};
        for (int j = 0; j < (b.ma + 1) / 2; ++j) w.p[j] = b.c.col(B_W, j);
        CHECK_HIP(gather_pairs(src, parts, b.ma, w, (const double*)b.s->M.ptr, b.c.N, b.c.st));
    } else {
        ColPtrs r{}, w{};
        for (int a = 0; a < b.ma; ++a) {
            r.p[a] = b.c.col(B_T1, b.act[a]);
            w.p[a] = b.c.col(B_W, a);
        }
        CHECK_HIP(precond(r, w, b.ma, (const double*)b.s->M.ptr, b.c.N, b.c.st));
    }
    return IWFPM_OK;
}

// W = T(R_A) with the learned map where it is in use (per instance), else
// M R_A (a batch's plain instances in one launch); sets b.lp_used
template <class Rt>
static int tall_precondition(Tall& t, std::vector<BInst>& in, const std::vector<int>& iter) {
    std::vector<int> plain;
    for (int i : iter) {
        BInst& b = in[i];
        b.lp_used = false;
        if (b.lp) {
            ColPtrs r{}, w{};
            int ncol = b.ma;
            if constexpr (Rt::real) {
                // R_A packed two per column into the (still free) HW buffer
                std::vector<RVec> Ract(b.ma);
                for (int a = 0; a < b.ma; ++a) Ract[a] = {b.c.col(B_T1, b.act[a] >> 1), b.act[a] & 1};
                unsigned long long parts = 0;
                const ColPtrs src = colptrs(Ract, &parts);
                ncol = (b.ma + 1) / 2;
                for (int j = 0; j < ncol; ++j) {
                    r.p[j] = b.c.col(B_HW, j);
                    w.p[j] = b.c.col(B_W, j);
                }
                CHECK_HIP(gather_pairs(src, parts, b.ma, r, nullptr, b.c.N, b.c.st));
            } else {
                for (int a = 0; a < b.ma; ++a) {
                    r.p[a] = b.c.col(B_T1, b.act[a]);
                    w.p[a] = b.c.col(B_W, a);
                }
            }
            if (learned_apply(b.lp, b.p, r, w, ncol, b.c.st) == IWFPM_OK) {
                b.lp_used = true;
                continue;
            }
            b.fallback = 1;
            b.lp = nullptr;
        }
        plain.push_back(i);
    }
    if (plain.empty()) return IWFPM_OK;
    if (t.single) {
        for (int i : plain)
            if (int rc = plain_precondition<Rt>(in[i])) return rc;
        return IWFPM_OK;
    }
    BatchOps& bo = t.bo;
    int blocks = 0, rc;
    if constexpr (Rt::real) {
        std::vector<GatherJob> jobs;
        for (int i : plain) {
            BInst& b = in[i];
            std::vector<RVec> Ract(b.ma);
            for (int a = 0; a < b.ma; ++a) Ract[a] = {b.c.col(B_T1, b.act[a] >> 1), b.act[a] & 1};
            GatherJob jb{};
            jb.src = colptrs(Ract, &jb.parts);
            jb.n = b.ma;
            jb.N = b.c.N;
            for (int j = 0; j < (b.ma + 1) / 2; ++j) jb.dst.p[j] = b.c.col(B_W, j);
            jb.M = (const double*)b.s->M.ptr;
            jb.nb = (int)std::min<long long>(1024, std::max<long long>(1, (jb.N + 255) / 256));
            jb.start = blocks;
            blocks += jb.nb;
            jobs.push_back(jb);
        }
        if ((rc = bo.wait_staged())) return rc;
        if ((rc = bo.reserve_host((void**)&bo.h_jobs, bo.jobs_cap, jobs.size() * sizeof(GatherJob)))) return rc;
        if ((rc = bo.reserve_dev(bo.d_jobs, jobs.size() * sizeof(GatherJob)))) return rc;
        std::memcpy(bo.h_jobs, jobs.data(), jobs.size() * sizeof(GatherJob));
        CHECK_HIP(
            hipMemcpyAsync(bo.d_jobs.ptr, bo.h_jobs, jobs.size() * sizeof(GatherJob), hipMemcpyHostToDevice, bo.st));
        CHECK_HIP(hipEventRecord(bo.staged, bo.st));
        CHECK_HIP(gather_pairs_batched((const GatherJob*)bo.d_jobs.ptr, (int)jobs.size(), blocks, bo.st));
    } else {
        std::vector<PreJob> jobs;
        for (int i : plain) {
            BInst& b = in[i];
            PreJob jb{};
            for (int a = 0; a < b.ma; ++a) {
                jb.R.p[a] = b.c.col(B_T1, b.act[a]);
                jb.W.p[a] = b.c.col(B_W, a);
            }
            jb.m = b.ma;
            jb.M = (const double*)b.s->M.ptr;
            jb.N = b.c.N;
            jb.nb = (int)std::min<long long>(1024, std::max<long long>(1, (jb.N + 255) / 256));
            jb.start = blocks;
            blocks += jb.nb;
            jobs.push_back(jb);
        }
        if ((rc = bo.wait_staged())) return rc;
        if ((rc = bo.reserve_host((void**)&bo.h_jobs, bo.jobs_cap, jobs.size() * sizeof(PreJob)))) return rc;
        if ((rc = bo.reserve_dev(bo.d_jobs, jobs.size() * sizeof(PreJob)))) return rc;
        std::memcpy(bo.h_jobs, jobs.data(), jobs.size() * sizeof(PreJob));
        CHECK_HIP(hipMemcpyAsync(bo.d_jobs.ptr, bo.h_jobs, jobs.size() * sizeof(PreJob), hipMemcpyHostToDevice, bo.st));
        CHECK_HIP(hipEventRecord(bo.staged, bo.st));
        CHECK_HIP(precond_batched((const PreJob*)bo.d_jobs.ptr, (int)jobs.size(), blocks, bo.st));
    }
    return IWFPM_OK;
}

// What a single solve adds: a start block, the Ritz vectors out, iterates
// captured for training the learned preconditioner, per-iteration lines.
struct SingleIO {
    const void* x0 = nullptr;  // N x m complex start block (complex route), or null
    void* evecs = nullptr;     // N x nev complex out, or null
    Capture* cap = nullptr;
};

template <class Rt>
static int lobpcg(int B, iwfpm_plan_s* const* plans, const iwfpm_eigs_opts& o, const SingleIO& io, double* evals,
                  double* eta_out, iwfpm_stats* stats, hipStream_t st) {
    const int nev = o.nev;
    const int m = o.block > 0 ? o.block : nev + std::max(2, nev / 4);
    if (m < nev || m > 32) return IWFPM_ERR_ARG;
    if (B > 1 && 3 * m > kMaxCols) return IWFPM_ERR_ARG;
    const bool explicit_ortho = force_explicit_ortho();
    const char* venv = std::getenv("IWFPM_VERBOSE");
    const bool verbose = B == 1 && venv && venv[0] == '1';
    std::vector<BInst> in(B);
    int rc;
    for (int i = 0; i < B; ++i) {
        BInst& b = in[i];
        b.p = plans[i];
        if (m > b.p->geom.N) return IWFPM_ERR_ARG;
        // block buffers of m trial vectors: m complex columns, or (m + 1) / 2
        // columns of real pairs
        if ((rc = solver_ensure(b.p, Rt::columns(m)))) return rc;
        int pk = o.precond == IWFPM_PRECOND_LEARNED ? IWFPM_PRECOND_PLAIN : o.precond;
        if ((rc = solver_precond(b.p, pk))) return rc;
        b.s = (Solver*)b.p->solver;
        b.c = Ctx{b.p, b.s, st, b.p->geom.N};
        b.prec = b.p->opts.precision;
        if (!b.p->sched[b.prec].ok) b.prec = 1 - b.prec;
        if (!b.p->sched[b.prec].ok) return IWFPM_ERR_UNSUPPORTED;
        b.can64 = b.p->sched[0].ok;
        b.hnorm = b.p->lam_max + b.p->vsum_abs;
        b.floor32 = 30.0 * 6e-8 * b.p->vsum_abs / b.hnorm;
        b.eta.assign(m, 1.0);
        if (o.precond == IWFPM_PRECOND_LEARNED) {
            b.lp = b.p->learned;
            if (!b.lp || !learned_ready(b.lp, b.p)) return IWFPM_ERR_WEIGHTS;
        }
    }
    Tall t;
    t.single = B == 1;
    t.bo.st = st;
    CHECK_HIP(hipEventCreateWithFlags(&t.bo.staged, hipEventDisableTiming));
    // a batch's applies: one batch object per convolution precision
    iwfpm_batch_t bat[2] = {nullptr, nullptr};
    struct BatchGuard {
        iwfpm_batch_t* b;
        ~BatchGuard() {
            for (int k = 0; k < 2; ++k)
                if (b[k]) iwfpm_batch_destroy(b[k]);
        }
    } bguard{bat};
    if (B > 1) {
        std::vector<iwfpm_plan_t> pl(plans, plans + B);
        for (int k = 0; k < 2; ++k) {
            bool ok = true;
            // plans on the five-pass schedule are applied one by one
            for (auto* p : pl) ok = ok && p->sched[k].ok && (p->sched[k].fused || p->sched[k].pd.split_mid == 0);
            if (ok && (rc = iwfpm_batch_create(B, pl.data(), k == 1 ? IWFPM_PREC_FP32 : IWFPM_PREC_FP64, 1, &bat[k])))
                return rc;
        }
    }
    auto V = [&](BInst& b, int buf, int v0, int cnt) { return Rt::vecs(b.c, buf, v0, cnt); };
    // H applied to the first cnt[i] trial vectors of bin into bout, by precision
    auto apply_all = [&](int bin, int bout, const std::vector<int>& cnt, const std::vector<int>& precs) -> int {
        for (int k = 0; k < 2; ++k) {
            std::vector<const void*> x(B, nullptr);
            std::vector<void*> y(B, nullptr);
            std::vector<int> nv(B, 0);
            bool any = false;
            for (int i = 0; i < B; ++i)
                if (cnt[i] > 0 && precs[i] == k) {
                    x[i] = in[i].c.col(bin, 0);
                    y[i] = in[i].c.col(bout, 0);
                    nv[i] = Rt::columns(cnt[i]);
                    in[i].matvecs += cnt[i];
                    any = true;
                }
            if (!any) continue;
            if (!bat[k]) {
                for (int i = 0; i < B; ++i)
                    if (nv[i] && (rc = plan_apply(in[i].p, x[i], y[i], nv[i], k, st))) return rc;
                continue;
            }
            if ((rc = iwfpm_batch_apply(bat[k], x.data(), y.data(), nv.data(), st))) return rc;
        }
        return IWFPM_OK;
    };
    // Rayleigh-Ritz on X alone (start blocks, blocks switched to float64, and
    // a last clean-up): X <- X C, HX <- HX C
    auto rr_blocks = [&](const std::vector<int>& which) -> int {
        if (which.empty()) return IWFPM_OK;
        std::vector<GramQ<Rt>> g;
        for (int i : which) {
            BInst& b = in[i];
            auto XHX = V(b, B_X, 0, m), HX = V(b, B_HX, 0, m);
            XHX.insert(XHX.end(), HX.begin(), HX.end());
            g.push_back({&b.c, V(b, B_X, 0, m), XHX});
        }
        std::vector<std::vector<cd>> G;
        if ((rc = tall_grams<Rt>(t, g, G))) return rc;
        std::vector<std::vector<cd>> C(which.size());
        std::vector<char> okt(which.size(), 1);
        parallel_for((int)which.size(), [&](int k) { okt[k] = rr_transform(G[k], m, in[which[k]].theta, C[k]); });
        for (char ok : okt)
            if (!ok) return IWFPM_ERR_NUMERIC;
        std::vector<LinQ<Rt>> l;
        for (size_t k = 0; k < which.size(); ++k) {
            BInst& b = in[which[k]];
            l.push_back({&b.c, V(b, B_X, 0, m), V(b, B_XN, 0, m), &C[k], m, 0.0});
            l.push_back({&b.c, V(b, B_HX, 0, m), V(b, B_HXN, 0, m), &C[k], m, 0.0});
        }
        if ((rc = tall_lincombs<Rt>(t, l))) return rc;
        for (int i : which) {
            std::swap(in[i].s->buf[B_X], in[i].s->buf[B_XN]);
            std::swap(in[i].s->buf[B_HX], in[i].s->buf[B_HXN]);
        }
        return IWFPM_OK;
    };

    // start blocks (seeded, or the caller's), orthonormalised
    for (int i = 0; i < B; ++i) {
        BInst& b = in[i];
        if (io.x0 && !Rt::real)
            CHECK_HIP(hipMemcpyAsync(b.c.col(B_X, 0), io.x0, (size_t)b.c.N * m * sizeof(double2),
                                     hipMemcpyDeviceToDevice, st));
        else
            CHECK_HIP(randn(b.c.col(B_X, 0), b.c.N * Rt::columns(m), o.seed + (unsigned long long)i, st));
    }
    {
        std::vector<GramQ<Rt>> g;
        for (auto& b : in) g.push_back({&b.c, V(b, B_X, 0, m), V(b, B_X, 0, m)});
        std::vector<std::vector<cd>> G;
        if ((rc = tall_grams<Rt>(t, g, G))) return rc;
        std::vector<int> bad(B, 0);
        parallel_for(B, [&](int i) {
            if (Rt::real) hermitian_part(G[i], m);
            bad[i] = svqb(G[i], m, in[i].T) < m;
        });
        for (int i = 0; i < B; ++i)
            if (bad[i]) return IWFPM_ERR_NUMERIC;
        std::vector<LinQ<Rt>> l;
        for (auto& b : in) l.push_back({&b.c, V(b, B_X, 0, m), V(b, B_XN, 0, m), &b.T, m, 0.0});
        if ((rc = tall_lincombs<Rt>(t, l))) return rc;
        for (auto& b : in) std::swap(b.s->buf[B_X], b.s->buf[B_XN]);
    }
    {
        std::vector<int> all_m(B, m), precs(B), allidx(B);
        for (int i = 0; i < B; ++i) {
            precs[i] = in[i].prec;
            allidx[i] = i;
        }
        if ((rc = apply_all(B_X, B_HX, all_m, precs))) return rc;
        if ((rc = rr_blocks(allidx))) return rc;
    }

    for (;;) {
        std::vector<int> live;
        for (int i = 0; i < B; ++i)
            if (!in[i].done) live.push_back(i);
        if (live.empty()) break;
        if ((rc = tall_residuals<Rt>(t, in, live, m))) return rc;
        if (io.cap) {
            // iterates (and residuals) for training the learned preconditioner
            Capture* cap = io.cap;
            BInst& b = in[0];
            if (!b.done && b.it > 0 && b.it % cap->stride == 0 && b.it != cap->last_it &&
                cap->got < (int)cap->X.size()) {
                const size_t bytes = (size_t)b.c.N * cap->ncol * sizeof(double2);
                CHECK_HIP(hipMemcpyAsync(cap->X[cap->got], b.c.col(B_X, 0), bytes, hipMemcpyDeviceToDevice, st));
                if (!cap->R.empty())
                    CHECK_HIP(hipMemcpyAsync(cap->R[cap->got], b.c.col(B_T1, 0), bytes, hipMemcpyDeviceToDevice, st));
                cap->eta.emplace_back(b.eta.begin(), b.eta.begin() + cap->ncol);
                cap->last_it = b.it;
                ++cap->got;
            }
        }
        // per-instance decisions
        std::vector<int> to64, iter, to_clean;
        for (int i : live) {
            BInst& b = in[i];
            if (b.done) continue;
            int conv = 0;
            double worst = 0.0;
            for (int j = 0; j < nev; ++j) {
                conv += b.eta[j] <= o.tol;
                worst = std::max(worst, b.eta[j]);
            }
            if (verbose)
                std::fprintf(stderr, "[iwfpm_eigs%s] it %d prec %s conv %d/%d worst_eta %.3e theta0 %.15g mp %d reortho %d\n",
                             Rt::real ? " real" : "", b.it, b.prec ? "fp32" : "fp64", conv, nev, worst, b.theta[0],
                             b.mp, b.reortho);
            if (conv == nev) {
                if ((b.prec == 0 || !b.can64) && b.cleaned) b.done = true;
                else if (b.prec == 0 || !b.can64) to_clean.push_back(i);  // re-orthonormalise X, take the pairs once more
                else to64.push_back(i);  // confirm with float64 applies
                if (!b.done) b.cleaned = true;
                continue;
            }
            if (b.it >= o.maxit) {
                b.done = true;
                b.status = IWFPM_ERR_NOCONV;
                continue;
            }
            // float32 convolution: continue with float64 applies once the
            // residuals reach its noise floor or stop improving
            bool stalled = false;
            if (worst < 0.5 * b.best_eta) {
                b.best_eta = worst;
                b.best_it = b.it;
            } else {
                stalled = worst < 1e-5 && b.it - b.best_it >= 20;
            }
            if (b.lp && b.it - b.best_it >= 50) {
                // learned preconditioner stagnating: continue with M
                b.fallback = 1;
                b.lp = nullptr;
                b.best_it = b.it;
            }
            if (b.prec == 1 && o.polish && b.can64 && (worst < b.floor32 || stalled)) {
                to64.push_back(i);
                continue;
            }
            iter.push_back(i);
        }
        if ((rc = rr_blocks(to_clean))) return rc;
        if (!to64.empty()) {
            std::vector<int> cx(B, 0), cp(B, 0), p0(B, 0);
            for (int i : to64) {
                in[i].prec = 0;
                in[i].best_eta = 1e300;
                cx[i] = m;
                cp[i] = in[i].mp;
            }
            if ((rc = apply_all(B_X, B_HX, cx, p0))) return rc;
            if ((rc = apply_all(B_P, B_HP, cp, p0))) return rc;
            if ((rc = rr_blocks(to64))) return rc;
        }
        if (iter.empty()) continue;
        for (int i : iter) {
            BInst& b = in[i];
            ++b.it;
            if (b.prec == 0 && b.p->opts.precision == 1) ++b.polished;
            // active set: the pairs not yet converged (soft locking)
            b.act.clear();
            for (int j = 0; j < m; ++j)
                if (b.eta[j] > o.tol) b.act.push_back(j);
            b.ma = (int)b.act.size();
            b.mq = b.mp;  // P: built last iteration from the then-active Ritz vectors, orthonormal and orthogonal to X
        }
        if ((rc = tall_precondition<Rt>(t, in, iter))) return rc;
        // W <- orthonormal basis of the part of W orthogonal to [X P]: one
        // explicit projection with the Gram [X P W]^H W, then the second
        // projection and SVQB in coefficient space (explicit twice as fallback)
        {
            std::vector<std::vector<typename Rt::V>> XPW(iter.size());
            std::vector<GramQ<Rt>> g;
            for (size_t k = 0; k < iter.size(); ++k) {
                BInst& b = in[iter[k]];
                XPW[k] = V(b, B_X, 0, m);
                auto P = V(b, B_P, 0, b.mq), Wv = V(b, B_W, 0, b.ma);
                XPW[k].insert(XPW[k].end(), P.begin(), P.end());
                XPW[k].insert(XPW[k].end(), Wv.begin(), Wv.end());
                g.push_back({&b.c, XPW[k], Wv});
            }
            std::vector<std::vector<cd>> Gall;
            if ((rc = tall_grams<Rt>(t, g, Gall))) return rc;
            // a non-finite learned direction falls back to M for the rest of the solve
            std::vector<GramQ<Rt>> again;
            std::vector<size_t> again_k;
            for (size_t k = 0; k < iter.size(); ++k) {
                BInst& b = in[iter[k]];
                if (!b.lp_used) continue;
                const int nx = m + b.mq;
                bool finite = true;
                for (int j = 0; j < b.ma; ++j)
                    finite = finite && std::isfinite(Gall[k][(size_t)(nx + j) + (size_t)j * (nx + b.ma)].real());
                if (finite) continue;
                b.fallback = 1;
                b.lp = nullptr;
                if ((rc = plain_precondition<Rt>(b))) return rc;
                again.push_back(g[k]);
                again_k.push_back(k);
            }
            if (!again.empty()) {
                std::vector<std::vector<cd>> G2;
                if ((rc = tall_grams<Rt>(t, again, G2))) return rc;
                for (size_t a = 0; a < again_k.size(); ++a) Gall[again_k[a]].swap(G2[a]);
            }
            std::vector<size_t> two(iter.size());
            for (size_t k = 0; k < iter.size(); ++k) two[k] = k;
            if (!explicit_ortho) {
                std::vector<std::vector<cd>> G1(two.size());
                std::vector<LinQ<Rt>> l1;
                std::vector<GramQ<Rt>> g2;
                for (size_t u = 0; u < two.size(); ++u) {
                    BInst& b = in[iter[two[u]]];
                    const int nx = m + b.mq;
                    G1[u] = neg_projection(Gall[two[u]], nx, b.ma);
                    std::vector<typename Rt::V> XP(XPW[two[u]].begin(), XPW[two[u]].begin() + nx);
                    l1.push_back({&b.c, XP, V(b, B_W, 0, b.ma), &G1[u], nx, 1.0});
                    g2.push_back({&b.c, XPW[two[u]], V(b, B_W, 0, b.ma)});
                }
                if ((rc = tall_lincombs<Rt>(t, l1))) return rc;
                std::vector<std::vector<cd>> Gall2;
                if ((rc = tall_grams<Rt>(t, g2, Gall2))) return rc;
                std::vector<char> ok2(two.size(), 0);
                std::vector<std::vector<cd>> Cm2(two.size());
                parallel_for((int)two.size(), [&](int u) {
                    BInst& b = in[iter[two[u]]];
                    ok2[u] = ortho_coefficients(Gall2[u], m + b.mq, b.ma, Cm2[u], b.mw);
                });
                std::vector<LinQ<Rt>> l2;
                std::vector<size_t> rest;
                for (size_t u = 0; u < two.size(); ++u) {
                    BInst& b = in[iter[two[u]]];
                    if (ok2[u])
                        l2.push_back({&b.c, XPW[two[u]], V(b, B_T1, 0, b.mw), &Cm2[u], m + b.mq + b.ma, 0.0});
                    else
                        rest.push_back(two[u]);
                }
                if ((rc = tall_lincombs<Rt>(t, l2))) return rc;
                two.swap(rest);
            }
            if (!two.empty()) {
                for (size_t k : two) ++in[iter[k]].reortho;
                for (int pass = 0; pass < 2; ++pass) {
                    std::vector<std::vector<typename Rt::V>> XP(two.size());
                    std::vector<GramQ<Rt>> g2;
                    for (size_t u = 0; u < two.size(); ++u) {
                        BInst& b = in[iter[two[u]]];
                        XP[u].assign(XPW[two[u]].begin(), XPW[two[u]].begin() + m + b.mq);
                        g2.push_back({&b.c, XP[u], V(b, B_W, 0, b.ma)});
                    }
                    std::vector<std::vector<cd>> G;
                    if ((rc = tall_grams<Rt>(t, g2, G))) return rc;
                    std::vector<LinQ<Rt>> l2;
                    for (size_t u = 0; u < two.size(); ++u) {
                        for (auto& v : G[u]) v = -v;
                        BInst& b = in[iter[two[u]]];
                        l2.push_back({&b.c, XP[u], V(b, B_W, 0, b.ma), &G[u], (int)XP[u].size(), 1.0});
                    }
                    if ((rc = tall_lincombs<Rt>(t, l2))) return rc;
                }
                std::vector<GramQ<Rt>> g2;
                for (size_t k : two) {
                    BInst& b = in[iter[k]];
                    g2.push_back({&b.c, V(b, B_W, 0, b.ma), V(b, B_W, 0, b.ma)});
                }
                std::vector<std::vector<cd>> G;
                if ((rc = tall_grams<Rt>(t, g2, G))) return rc;
                parallel_for((int)two.size(), [&](int u) {
                    BInst& b = in[iter[two[u]]];
                    if (Rt::real) hermitian_part(G[u], b.ma);
                    b.mw = svqb(G[u], b.ma, b.T, 1e-10);
                });
                std::vector<LinQ<Rt>> l2;
                for (size_t k : two) {
                    BInst& b = in[iter[k]];
                    l2.push_back({&b.c, V(b, B_W, 0, b.ma), V(b, B_T1, 0, b.mw), &b.T, b.ma, 0.0});
                }
                if ((rc = tall_lincombs<Rt>(t, l2))) return rc;
            }
            for (int i : iter) std::swap(in[i].s->buf[B_W], in[i].s->buf[B_T1]);
        }
        // HW = H W
        {
            std::vector<int> cnt(B, 0), pr(B, 0);
            for (int i : iter) {
                cnt[i] = in[i].mw;
                pr[i] = in[i].prec;
            }
            if ((rc = apply_all(B_W, B_HW, cnt, pr))) return rc;
        }
        // Rayleigh-Ritz on the orthonormal basis S = [X W P]: with
        // X^H H X = diag(theta) only S^H [HW HP] is formed; the small problems
        // on host threads
        std::vector<std::vector<typename Rt::V>> S(iter.size()), HS(iter.size());
        {
            std::vector<GramQ<Rt>> g;
            for (size_t k = 0; k < iter.size(); ++k) {
                BInst& b = in[iter[k]];
                S[k] = V(b, B_X, 0, m);
                HS[k] = V(b, B_HX, 0, m);
                auto Wn = V(b, B_W, 0, b.mw), HWn = V(b, B_HW, 0, b.mw);
                auto Pn = V(b, B_P, 0, b.mq), HPn = V(b, B_HP, 0, b.mq);
                S[k].insert(S[k].end(), Wn.begin(), Wn.end());
                HS[k].insert(HS[k].end(), HWn.begin(), HWn.end());
                S[k].insert(S[k].end(), Pn.begin(), Pn.end());
                HS[k].insert(HS[k].end(), HPn.begin(), HPn.end());
                b.ns = (int)S[k].size();
                g.push_back({&b.c, S[k], std::vector<typename Rt::V>(HS[k].begin() + m, HS[k].end())});
            }
            std::vector<std::vector<cd>> G;
            if ((rc = tall_grams<Rt>(t, g, G))) return rc;
            parallel_for((int)iter.size(), [&](int k) {
                BInst& b = in[iter[k]];
                b.mpn = rr_coefficients(G[k], b.theta, m, b.ns, b.act, b.th, b.U);
            });
        }
        // [X_new | P_new] = S U, [HX_new | HP_new] = HS U
        {
            std::vector<LinQ<Rt>> l;
            for (size_t k = 0; k < iter.size(); ++k) {
                BInst& b = in[iter[k]];
                auto out = V(b, B_XN, 0, m), hout = V(b, B_HXN, 0, m);
                auto pn = V(b, B_PN, 0, b.mpn), hpn = V(b, B_HPN, 0, b.mpn);
                out.insert(out.end(), pn.begin(), pn.end());
                hout.insert(hout.end(), hpn.begin(), hpn.end());
                l.push_back({&b.c, S[k], out, &b.U, b.ns, 0.0});
                l.push_back({&b.c, HS[k], hout, &b.U, b.ns, 0.0});
            }
            if ((rc = tall_lincombs<Rt>(t, l))) return rc;
            for (int i : iter) {
                BInst& b = in[i];
                std::swap(b.s->buf[B_X], b.s->buf[B_XN]);
                std::swap(b.s->buf[B_HX], b.s->buf[B_HXN]);
                std::swap(b.s->buf[B_P], b.s->buf[B_PN]);
                std::swap(b.s->buf[B_HP], b.s->buf[B_HPN]);
                b.mp = b.mpn;
                b.theta.assign(b.th.begin(), b.th.begin() + m);
            }
        }
    }
    if (io.evecs) {
        BInst& b = in[0];
        if constexpr (Rt::real) {
            unsigned long long parts = 0;
            const ColPtrs src = colptrs(rvecs(b.c, B_X, 0, nev), &parts);
            ColPtrs dst{};
            for (int j = 0; j < nev; ++j) dst.p[j] = (double2*)io.evecs + (size_t)j * b.c.N;
            CHECK_HIP(unpack_real(src, parts, nev, dst, b.c.N, st));
        } else {
            CHECK_HIP(hipMemcpyAsync(io.evecs, b.c.col(B_X, 0), (size_t)b.c.N * nev * sizeof(double2),
                                     hipMemcpyDeviceToDevice, st));
        }
    }
    CHECK_HIP(hipStreamSynchronize(st));
    int worst_status = IWFPM_OK;
    for (int i = 0; i < B; ++i) {
        BInst& b = in[i];
        for (int j = 0; j < nev; ++j) {
            evals[(size_t)i * nev + j] = b.theta[j];
            if (eta_out) eta_out[(size_t)i * nev + j] = b.eta[j];
        }
        if (stats) {
            iwfpm_stats& s = stats[i];
            s.iterations = b.it;
            s.restarts = 0;
            s.matvecs = b.matvecs;
            s.polished = b.polished;
            s.fallback = b.fallback;
            int conv = 0;
            for (int j = 0; j < nev; ++j) conv += b.eta[j] <= o.tol;
            s.converged = conv;
        }
        if (b.status != IWFPM_OK && worst_status == IWFPM_OK) worst_status = b.status;
    }
    return worst_status;
}

int eigs_capture(iwfpm_plan_s* p, const iwfpm_eigs_opts& o, Capture* cap, double* evals, void* evecs,
                 hipStream_t st) {
    if (o.nev < 1 || o.nev > p->geom.N || !cap || cap->ncol > o.nev) return IWFPM_ERR_ARG;
    SingleIO io;
    io.evecs = evecs;
    io.cap = cap;
    return lobpcg<CplxRoute>(1, &p, o, io, evals, nullptr, nullptr, st);
}

}  // namespace iwfpm

using namespace iwfpm;

extern "C" {

void iwfpm_default_eigs_opts(iwfpm_eigs_opts* o) {
    if (!o) return;
    o->nev = 8;
    o->block = 0;
    o->tol = 1e-8;
    o->maxit = 1000;
    o->precond = IWFPM_PRECOND_PLAIN;
    o->seed = 2404045070ull;
    o->polish = 1;
    o->arith = 0;
}

int iwfpm_eigs(iwfpm_plan_t p, const iwfpm_eigs_opts* opts, const void* x0, double* evals, void* evecs, double* eta,
               iwfpm_stats* stats, void* stream) {
    if (!p || !opts || !evals) return IWFPM_ERR_ARG;
    if (opts->nev < 1 || opts->nev > p->geom.N || !(opts->tol > 0.0) || opts->maxit < 0) return IWFPM_ERR_ARG;
    if (opts->precond < 0 || opts->precond > 2) return IWFPM_ERR_ARG;
    if (p->host_only) return IWFPM_ERR_NODEVICE;
    DeviceGuard guard(p->opts.device);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    if (opts->arith < 0 || opts->arith > 2) return IWFPM_ERR_ARG;
    const bool real = opts->arith == 2 || (opts->arith == 0 && !x0 && real_symmetric(p));
    if (real && (x0 || !real_symmetric(p))) return IWFPM_ERR_ARG;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    auto t0 = std::chrono::steady_clock::now();
    SingleIO io;
    io.x0 = x0;
    io.evecs = evecs;
    int rc = real ? lobpcg<RealRoute>(1, &p, *opts, io, evals, eta, stats, (hipStream_t)stream)
                  : lobpcg<CplxRoute>(1, &p, *opts, io, evals, eta, stats, (hipStream_t)stream);
    if (stats) stats->t_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int iwfpm_eigs_batched(int B, const iwfpm_plan_t* plans, const iwfpm_eigs_opts* opts, double* evals, double* eta,
                       iwfpm_stats* stats, void* stream) {
    if (B < 1 || !plans || !opts || !evals) return IWFPM_ERR_ARG;
    if (opts->nev < 1 || !(opts->tol > 0.0) || opts->maxit < 0) return IWFPM_ERR_ARG;
    int dev = -1;
    for (int i = 0; i < B; ++i) {
        if (!plans[i]) return IWFPM_ERR_ARG;
        if (plans[i]->host_only) return IWFPM_ERR_NODEVICE;
        if (dev < 0) dev = plans[i]->opts.device;
        if (plans[i]->opts.device != dev) return IWFPM_ERR_ARG;
        if (opts->nev > plans[i]->geom.N) return IWFPM_ERR_ARG;
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return IWFPM_ERR_ARG;
    }
    if (opts->arith < 0 || opts->arith > 2) return IWFPM_ERR_ARG;
    bool all_real = true;
    for (int i = 0; i < B; ++i) all_real = all_real && real_symmetric(plans[i]);
    const bool real = opts->arith == 2 || (opts->arith == 0 && all_real);
    if (real && !all_real) return IWFPM_ERR_ARG;
    DeviceGuard guard(dev);
    if (!guard.ok) return IWFPM_ERR_DEVICE;
    if (stats) std::memset(stats, 0, sizeof(iwfpm_stats) * B);
    auto t0 = std::chrono::steady_clock::now();
    int rc = real ? lobpcg<RealRoute>(B, plans, *opts, SingleIO{}, evals, eta, stats, (hipStream_t)stream)
                  : lobpcg<CplxRoute>(B, plans, *opts, SingleIO{}, evals, eta, stats, (hipStream_t)stream);
    double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats)
        for (int i = 0; i < B; ++i) stats[i].t_total = t;
    return rc;
}

int iwfpm_dense_geneig(int n, const double* A, const double* B, double* w, double* C) {
    if (n < 1 || n > 512 || !A || !w || !C) return IWFPM_ERR_ARG;
    std::vector<cd> a((size_t)n * n), b((size_t)n * n, 0.0), c;
    for (size_t i = 0; i < a.size(); ++i) a[i] = cd(A[2 * i], A[2 * i + 1]);
    if (B)
        for (size_t i = 0; i < b.size(); ++i) b[i] = cd(B[2 * i], B[2 * i + 1]);
    else
        for (int i = 0; i < n; ++i) b[i + (size_t)i * n] = 1.0;
    std::vector<double> th;
    if (!gen_eigh(a, b, n, th, c)) return IWFPM_ERR_NUMERIC;
    for (int i = 0; i < n; ++i) w[i] = th[i];
    for (size_t i = 0; i < c.size(); ++i) {
        C[2 * i] = c[i].real();
        C[2 * i + 1] = c[i].imag();
    }
    return IWFPM_OK;
}

int iwfpm_dense_heev_lowest(int n, int nv, const double* A, double* w, double* V) {
    if (n < 1 || n > 512 || nv < 0 || nv > n || !A || !w || (nv > 0 && !V)) return IWFPM_ERR_ARG;
    std::vector<cd> a((size_t)n * n), v;
    for (size_t i = 0; i < a.size(); ++i) a[i] = cd(A[2 * i], A[2 * i + 1]);
    std::vector<double> th;
    if (!heev_lowest(a, n, nv, th, v)) heev(a, n, th, v);
    for (int i = 0; i < n; ++i) w[i] = th[i];
    for (size_t i = 0; i < (size_t)n * nv; ++i) {
        V[2 * i] = v[i].real();
        V[2 * i + 1] = v[i].imag();
    }
    return IWFPM_OK;
}

int iwfpm_dense_svqb(int k, const double* G, double* T, int* rank) {
    if (k < 1 || k > 512 || !G || !T || !rank) return IWFPM_ERR_ARG;
    std::vector<cd> g((size_t)k * k), t;
    for (size_t i = 0; i < g.size(); ++i) g[i] = cd(G[2 * i], G[2 * i + 1]);
    *rank = svqb(g, k, t);
    for (size_t i = 0; i < t.size(); ++i) {
        T[2 * i] = t[i].real();
        T[2 * i + 1] = t[i].imag();
    }
    return IWFPM_OK;
}

int iwfpm_destroy(iwfpm_plan_t p) {
    if (!p) return IWFPM_ERR_ARG;
    if (!p->host_only) {
        DeviceGuard g(p->opts.device);
        (void)hipDeviceSynchronize();
        dev_free(p->d_slice_a);
        dev_free(p->d_slice_g);
        dev_free(p->d_vtab32);
        dev_free(p->d_vtab64);
        dev_free(p->d_vgrid32);
        dev_free(p->d_vgrid64);
        dev_free(p->d_tw32);
        dev_free(p->d_tw64);
        dev_free(p->d_ws);
        dev_free(p->d_ef_freq);
        dev_free(p->d_ef_ws);
        for (auto& sl : p->prof.ring)
            for (auto& e : sl.ev)
                if (e) (void)hipEventDestroy(e);
        solver_free((Solver*)p->solver);
        learned_free(p->learned);
    }
    delete p;
    return IWFPM_OK;
}

}  // extern "C"
