"""Plain, slow CPU oracle of the irrational-window-filter projection method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this module: only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code, tables or constants with the HIP
library; it is written from the paper's definitions in float64/complex128.

Conventions (Sec. 2, Def. 2.1-2.2; Sec. 3.1-3.3 of the paper):

* ``P`` is d x n with the kinetic energy of mode k equal to 1/2 |2 pi P k|^2.
  The paper's own examples carry the 2 pi inside P; pass P_paper / (2 pi).
* ``K`` (length d) and ``L`` (length n-d) give the window W_{K,L}: k_II in
  [-L, L)^{n-d} and k_I + Q k_II in [-K, K)^d with Q = P_I^{-1} P_II (Sec. 3.1).
* The lifted grid K*_{K,L} = [0,2K)^d x [0,2L)^{n-d} (Sec. 3.2) is stored as
  a row-major array whose axes are (k_{d+1}, ..., k_n, k_1, ..., k_d): the
  k_II axes are slow and the k_I axes are fast.  "Grid order" below means the
  flat index of that array.
* The potential is given by its parent-function Fourier modes: integer
  vectors m (paper order, length n) with coefficients Vhat_m.

Each function cites the passage it follows.  The ``variant`` argument selects
how the sheared offset q = Q k_II enters the window:
  ``"exact"``   q itself (the window as defined in Sec. 3.1),
  ``"rounded"`` floor(q + 1/2) (the reading under which Table 1's
                condition numbers of H are reproduced),
  ``"pm"``      0, i.e. the shear switched off, which is the projection
                method's rectangle [-K,K)^d x [-L,L)^{n-d} (Sec. 2, Sec. 4).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------------------
# Sec. 3.1: splitting P and the sheared offset
# ---------------------------------------------------------------------------

def split_projection(P: np.ndarray, d: int) -> np.ndarray:
    """Q = P_I^{-1} P_II with P = (P_I, P_II), P_I the leading d x d block (Sec. 3.1)."""
    P = np.asarray(P, dtype=np.float64)
    P_I = P[:, :d]
    P_II = P[:, d:]
    return sla.solve(P_I, P_II)


def sheared_offset(Q: np.ndarray, k_II: np.ndarray) -> np.ndarray:
    """q = Q k_II for each row of k_II, formed as plain products and sums.

    Written as separate multiplies and adds (no fused multiply-add, no BLAS)
    so that cancelling terms such as c*k - c*k give an exact zero.
    """
    k_II = np.atleast_2d(k_II).astype(np.float64)
    d, nd = Q.shape
    q = np.zeros((k_II.shape[0], d))
    for j in range(d):
        acc = np.zeros(k_II.shape[0])
        for i in range(nd):
            acc = acc + Q[j, i] * k_II[:, i]
        q[:, j] = acc
    return q


def effective_offset(q: np.ndarray, variant: str) -> np.ndarray:
    """The offset the window is sheared by, per the variant described above."""
    if variant == "exact":
        return q
    if variant == "rounded":
        return np.floor(q + 0.5)
    if variant == "pm":
        return np.zeros_like(q)
    raise ValueError(f"unknown window variant {variant!r}")


# ---------------------------------------------------------------------------
# Sec. 3.2: the lifted grid, the index-shift map and its inverse
# ---------------------------------------------------------------------------

def grid_extents(K, L) -> tuple:
    """Array shape of K*_{K,L}: (2L_1, ..., 2L_{n-d}, 2K_1, ..., 2K_d)."""
    return tuple(2 * int(x) for x in L) + tuple(2 * int(x) for x in K)


def grid_kstar(K, L) -> np.ndarray:
    """k* in paper order (k*_1..k*_n) for every grid position, in grid order."""
    d, nd = len(K), len(L)
    shape = grid_extents(K, L)
    idx = np.indices(shape).reshape(len(shape), -1).T  # array-axis order
    kstar = np.empty_like(idx)
    kstar[:, :d] = idx[:, nd:]
    kstar[:, d:] = idx[:, :nd]
    return kstar


def kstar_to_position(kstar: np.ndarray, K, L) -> np.ndarray:
    """Flat grid-order index of paper-order k* rows."""
    d, nd = len(K), len(L)
    shape = grid_extents(K, L)
    axes = np.concatenate([kstar[:, d:], kstar[:, :d]], axis=1)
    return np.ravel_multi_index(tuple(axes.T), shape)


def index_shift(k: np.ndarray, K, L) -> np.ndarray:
    """The index-shift map rho of eq:index mod: k_j mod 2K (j<=d), k_j mod 2L (j>d)."""
    k = np.atleast_2d(k)
    d = len(K)
    mods = np.array([2 * x for x in K] + [2 * x for x in L])
    out = np.mod(k, mods)
    assert out.shape[1] == d + len(L)
    return out


def inverse_index_shift(kstar: np.ndarray, Q: np.ndarray, K, L, variant="exact") -> np.ndarray:
    """rho^{-1}(k*) following eq:inverse1-eq:inverse3, in that order.

    Step 1 (eq:inverse2): k_II from k*_II.
    Step 2 (eq:inverse3): with R_j = ceil((-K - (Q k_II)_j) / 2K) * 2K,
    k_j = k*_j + R_j if k*_j + R_j + (Q k_II)_j < K, else k*_j + R_j - 2K.
    """
    kstar = np.atleast_2d(kstar).astype(np.int64)
    d, nd = len(K), len(L)
    k = np.empty_like(kstar)
    for jj in range(nd):
        Lj = int(L[jj])
        ks = kstar[:, d + jj]
        k[:, d + jj] = np.where(ks < Lj, ks, ks - 2 * Lj)
    q = effective_offset(sheared_offset(Q, k[:, d:]), variant)
    for j in range(d):
        Kj = int(K[j])
        R = np.ceil((-Kj - q[:, j]) / (2 * Kj)) * (2 * Kj)
        t = kstar[:, j] + R
        kj = np.where(t + q[:, j] < Kj, t, t - 2 * Kj)
        k[:, j] = kj.astype(np.int64)
    return k


def grid_labels(P, d: int, K, L, variant="exact") -> np.ndarray:
    """True indices k = rho^{-1}(k*) (paper order) for every grid position, grid order."""
    Q = split_projection(P, d)
    return inverse_index_shift(grid_kstar(K, L), Q, K, L, variant)


def window_points_bruteforce(P, d: int, K, L, variant="exact") -> np.ndarray:
    """Enumerate K_{K,L} = W_{K,L} intersected with Z^n (eq:non-tensor) by scanning.

    For every k_II in [-L, L)^{n-d}, every integer k_I in a generous box is
    tested against k_I + q in [-K, K).  Slow; for small windows only.
    """
    Q = split_projection(P, d)
    nd = len(L)
    ranges = [range(-int(x), int(x)) for x in L]
    pts = []
    for kII in np.array(np.meshgrid(*ranges, indexing="ij")).reshape(nd, -1).T:
        q = effective_offset(sheared_offset(Q, kII[None, :]), variant)[0]
        lo = [int(math.floor(-K[j] - q[j])) - 1 for j in range(d)]
        hi = [int(math.ceil(K[j] - q[j])) + 1 for j in range(d)]
        for kI in np.array(np.meshgrid(*[range(lo[j], hi[j] + 1) for j in range(d)],
                                       indexing="ij")).reshape(d, -1).T:
            z = kI + q
            if np.all(z >= -np.asarray(K)) and np.all(z < np.asarray(K)):
                pts.append(np.concatenate([kI, kII]))
    return np.array(pts, dtype=np.int64)


# ---------------------------------------------------------------------------
# Sec. 4.1: the discretised Hamiltonian  H = Lambda + F V F^{-1}
# ---------------------------------------------------------------------------

def kinetic(P, k: np.ndarray) -> np.ndarray:
    """Lambda = 1/2 |2 pi P k|^2 per row of k (Sec. 4.1, with 2 pi taken out of P)."""
    P = np.asarray(P, dtype=np.float64)
    k = np.atleast_2d(k).astype(np.float64)
    d, n = P.shape
    tot = np.zeros(k.shape[0])
    for j in range(d):
        acc = np.zeros(k.shape[0])
        for i in range(n):
            acc = acc + P[j, i] * k[:, i]
        g = TWO_PI * acc
        tot = tot + g * g
    return 0.5 * tot


def check_modes(modes, vhat, n: int):
    """Validate a mode list: integer n-vectors and V_{-m} = conj(V_m) (real potential)."""
    modes = np.asarray(modes, dtype=np.int64).reshape(-1, n)
    vhat = np.asarray(vhat, dtype=np.complex128).reshape(-1)
    lookup = {tuple(m): v for m, v in zip(modes, vhat)}
    for m, v in lookup.items():
        mm = tuple(-x for x in m)
        if mm not in lookup or abs(lookup[mm] - np.conj(v)) > 1e-14 * max(1.0, abs(v)):
            raise ValueError(f"potential is not real: mode {m} has no conjugate partner")
    return modes, vhat


def convolution_sparse(K, L, modes, vhat) -> sp.csr_matrix:
    """The potential block F V F^{-1} as the wrapped convolution it equals.

    By the discrete orthogonality of Appendix C (the aliasing identity), the
    product of two grid functions has coefficient sum_m Vhat_m psi[k* - m] with
    the index taken modulo the grid extents, so
        (C psi)[k*] = sum_m Vhat_m psi[(k* - m) mod ext].
    """
    n = len(K) + len(L)
    modes, vhat = check_modes(modes, vhat, n)
    kstar = grid_kstar(K, L)
    N = kstar.shape[0]
    mods = np.array([2 * x for x in K] + [2 * x for x in L])
    rows, cols, vals = [], [], []
    src = np.arange(N)
    for m, v in zip(modes, vhat):
        tgt = kstar_to_position(np.mod(kstar + m[None, :], mods), K, L)
        rows.append(tgt)
        cols.append(src)
        vals.append(np.full(N, v))
    if not vals:
        return sp.csr_matrix((N, N), dtype=np.complex128)
    C = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N)).tocsr()
    C.sum_duplicates()
    return C


def hamiltonian_sparse(P, d: int, K, L, modes, vhat, variant="exact") -> sp.csr_matrix:
    """H = diag(Lambda) + C on the lifted grid, grid order (Sec. 4.1)."""
    k = grid_labels(P, d, K, L, variant)
    lam = kinetic(P, k)
    C = convolution_sparse(K, L, modes, vhat)
    return (sp.diags(lam.astype(np.complex128)) + C).tocsr()


def hamiltonian_dense(P, d, K, L, modes, vhat, variant="exact") -> np.ndarray:
    return hamiltonian_sparse(P, d, K, L, modes, vhat, variant).toarray()


def apply(P, d, K, L, modes, vhat, psi, variant="exact") -> np.ndarray:
    """H psi for a block of columns psi (N x m, grid order)."""
    H = hamiltonian_sparse(P, d, K, L, modes, vhat, variant)
    return H @ np.asarray(psi, dtype=np.complex128)


def apply_points(P, d, K, L, modes, vhat, psi, positions, variant="exact") -> np.ndarray:
    """(H psi)[i] for selected grid positions only, one by one (for large grids)."""
    n = len(K) + len(L)
    modes, vhat = check_modes(modes, vhat, n)
    Q = split_projection(P, d)
    positions = np.asarray(positions, dtype=np.int64)
    shape = grid_extents(K, L)
    nd = len(L)
    axes = np.array(np.unravel_index(positions, shape)).T
    kstar = np.concatenate([axes[:, nd:], axes[:, :nd]], axis=1)
    k = inverse_index_shift(kstar, Q, K, L, variant)
    lam = kinetic(P, k)
    mods = np.array([2 * x for x in K] + [2 * x for x in L])
    psi = np.asarray(psi)
    out = lam[:, None] * psi[positions]
    for m, v in zip(modes, vhat):
        src = kstar_to_position(np.mod(kstar - m[None, :], mods), K, L)
        out = out + v * psi[src]
    return out


def apply_shifts(P, d, K, L, modes, vhat, psi, variant="exact") -> np.ndarray:
    """H psi for a block of columns psi (N x m, grid order) without forming H:
    Lambda psi plus the wrapped convolution written as cyclic shifts of the
    grid array, (C psi)[k*] = sum_m Vhat_m psi[(k* - m) mod ext] (Sec. 4.1;
    the aliasing identity of Appendix C).  One column at a time, so memory
    stays at a few copies of one vector even on the 16^6 grid."""
    n = len(K) + len(L)
    modes, vhat = check_modes(modes, vhat, n)
    d_, nd = len(K), len(L)
    shape = grid_extents(K, L)
    lam = kinetic(P, grid_labels(P, d, K, L, variant))
    psi = np.asarray(psi, dtype=np.complex128)
    cols = psi.reshape(psi.shape[0], -1)
    out = np.empty_like(cols)
    # paper index j of a mode -> axis of the grid array (k_II axes first)
    axis = [nd + j if j < d_ else j - d_ for j in range(n)]
    for c in range(cols.shape[1]):
        x = cols[:, c].reshape(shape)
        y = lam.reshape(shape) * x
        for m, v in zip(modes, vhat):
            y = y + v * np.roll(x, shift=tuple(int(t) for t in m), axis=tuple(axis))
        out[:, c] = y.reshape(-1)
    return out.reshape(psi.shape)


# ---------------------------------------------------------------------------
# Sec. 3.3: the same operator through explicit DFT matrices (F = T F*)
# ---------------------------------------------------------------------------

def potential_on_grid(K, L, modes, vhat) -> np.ndarray:
    """V(y_l) = sum_m Vhat_m exp(i m . y_l) on G_{K,L} (eq:G_KL), grid order."""
    n = len(K) + len(L)
    modes, vhat = check_modes(modes, vhat, n)
    ell = grid_kstar(K, L)  # the grid multi-index l has the same range as k*
    ext = np.array([2 * x for x in K] + [2 * x for x in L], dtype=np.float64)
    y = TWO_PI * ell / ext[None, :]
    V = np.zeros(ell.shape[0], dtype=np.complex128)
    for m, v in zip(modes, vhat):
        V = V + v * np.exp(1j * (y @ m.astype(np.float64)))
    return V


def dft_matrices(P, d, K, L, variant="exact"):
    """Explicit transforms between coefficients and grid values.

    Returns (Finv, F) where Finv[l, i] = exp(i k_i . y_l) maps coefficient
    vectors (grid order, labelled by the true k_i = rho^{-1}(k*_i)) to values
    U(y_l), and F = Finv^H / N realises the discrete inner product
    eq:new_inner_product.  Using the true labels k rather than k* exercises
    eq:basis_equivalent: both give the same matrix.
    """
    k = grid_labels(P, d, K, L, variant).astype(np.float64)
    ell = grid_kstar(K, L).astype(np.float64)
    ext = np.array([2 * x for x in K] + [2 * x for x in L], dtype=np.float64)
    y = TWO_PI * ell / ext[None, :]
    Finv = np.exp(1j * (y @ k.T))
    N = Finv.shape[0]
    F = Finv.conj().T / N
    return Finv, F


def hamiltonian_via_dft(P, d, K, L, modes, vhat, variant="exact") -> np.ndarray:
    """Lambda + F diag(V) F^{-1} with dense DFT matrices (Sec. 4.1, eq:F)."""
    k = grid_labels(P, d, K, L, variant)
    lam = kinetic(P, k)
    Finv, F = dft_matrices(P, d, K, L, variant)
    V = potential_on_grid(K, L, modes, vhat)
    return np.diag(lam).astype(np.complex128) + F @ (V[:, None] * Finv)


def fft_apply_setup(P, d, K, L, modes, vhat, variant="exact"):
    """Alg. 1's set-up for the host FFT route: the kinetic diagonal with the
    true labels and the potential on G_{K,L}.  Returns (grid shape, Lambda,
    V on the grid)."""
    shape = grid_extents(K, L)
    lam = kinetic(P, grid_labels(P, d, K, L, variant))
    V = potential_on_grid(K, L, modes, vhat).reshape(shape)
    return shape, lam, V


def apply_fft_prepared(setup, psi, workers: int = 1) -> np.ndarray:
    """H psi by Alg. 1's route on the host: the coefficients (grid order, i.e.
    already relabelled by T) go to grid values by the inverse DFT, are
    multiplied by V(y_l), and return by the forward DFT; the kinetic diagonal
    is added with the true labels (Sec. 3.3 and Sec. 4.1, eq:F).  With
    numpy's conventions ifftn carries the 1/N and fftn none, and
    u(y_l) = N ifftn(psi), so the potential block is fftn(V * ifftn(psi)).
    ``workers`` is passed to scipy.fft (threads over the batch of columns)."""
    import scipy.fft as sfft
    shape, lam, V = setup
    psi = np.asarray(psi, dtype=np.complex128)
    cols = psi.reshape(psi.shape[0], -1)
    m = cols.shape[1]
    axes = tuple(range(1, len(shape) + 1))
    g = cols.T.reshape((m,) + shape)
    u = sfft.ifftn(g, axes=axes, workers=workers)
    u *= V[None]
    c = sfft.fftn(u, axes=axes, workers=workers).reshape(m, -1).T
    return (lam[:, None] * cols + c).reshape(psi.shape)


def apply_fft(P, d, K, L, modes, vhat, psi, variant="exact", workers: int = 1) -> np.ndarray:
    """H psi by the host FFT route (set-up and apply, see apply_fft_prepared)."""
    return apply_fft_prepared(fft_apply_setup(P, d, K, L, modes, vhat, variant), psi, workers)


def discrete_inner_product(K, L, U_vals, V_vals) -> complex:
    """<U, V>_{K,L} of eq:new_inner_product from grid values."""
    N = U_vals.shape[0]
    return np.sum(U_vals * np.conj(V_vals)) / N


# ---------------------------------------------------------------------------
# eq:precond: the diagonal preconditioner
# ---------------------------------------------------------------------------

def preconditioner_definition(H: np.ndarray) -> np.ndarray:
    """M_ii = h_ii / ||H e_i||_2^2, the column-norm form of eq:precond (dense H)."""
    H = np.asarray(H)
    col = np.sum(np.abs(H) ** 2, axis=0)
    return np.real(np.diag(H)) / col


def preconditioner_sparse(H: sp.spmatrix) -> np.ndarray:
    """Same as preconditioner_definition for a sparse H (column norms of CSR)."""
    Hc = sp.csc_matrix(H)
    col = np.asarray(abs(Hc).power(2).sum(axis=0)).ravel()
    return np.real(Hc.diagonal()) / col


# ---------------------------------------------------------------------------
# Eigenpairs
# ---------------------------------------------------------------------------

def eigs_dense(H: np.ndarray, nev: int):
    """Lowest nev eigenpairs of a dense Hermitian H (LAPACK)."""
    w, v = sla.eigh(H, subset_by_index=[0, nev - 1])
    return w, v


def backward_error(H, X: np.ndarray, theta: np.ndarray, hnorm: float) -> np.ndarray:
    """eta_i = ||H x_i - theta_i x_i|| / ((||H|| + |theta_i|) ||x_i||)."""
    R = H @ X - X * theta[None, :]
    return np.linalg.norm(R, axis=0) / ((hnorm + np.abs(theta)) * np.linalg.norm(X, axis=0))


def norm_bound(P, d, K, L, modes, vhat, variant="exact") -> float:
    """max Lambda + sum |Vhat_m|, an upper bound of ||H||_2."""
    k = grid_labels(P, d, K, L, variant)
    return float(np.max(kinetic(P, k)) + np.sum(np.abs(np.asarray(vhat))))


def eigs_sparse(H: sp.spmatrix, nev: int, tol: float = 1e-10, maxiter: int = 2000,
                X0: np.ndarray | None = None, seed: int = 0, block: int | None = None,
                shift: float | None = None):
    """Lowest nev eigenpairs of a sparse Hermitian H with scipy's LOBPCG.

    Preconditioned by eq:precond applied to H + sigma I, where sigma (if not
    given) makes the diagonal positive: sigma = max(0, 1 - min diag(H)) + ...
    """
    N = H.shape[0]
    m = block or (nev + max(4, nev // 4))
    if X0 is None:
        rng = np.random.default_rng(seed)
        X0 = rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m))
    diag = np.real(H.diagonal())
    if shift is None:
        shift = max(0.0, 1.0 - float(diag.min()))
    Hs = (H + shift * sp.identity(N, format="csr")).tocsr()
    Mdiag = preconditioner_sparse(Hs)
    Mop = spla.LinearOperator((N, N), matvec=lambda x: Mdiag * x.ravel() if x.ndim == 1 else Mdiag[:, None] * x,
                              matmat=lambda X: Mdiag[:, None] * X, dtype=np.complex128)
    w, v = spla.lobpcg(Hs, X0, M=Mop, tol=tol, maxiter=maxiter, largest=False)
    order = np.argsort(w)
    w = w[order][:nev] - shift
    v = v[:, order][:, :nev]
    return w, v


# ---------------------------------------------------------------------------
# eq:int and Alg. 1 (final step): the eigenfunction in physical space, and the
# error measures of Sec. 4 (numerical experiments)
# ---------------------------------------------------------------------------

def observation_axes(origin, step, npts) -> list:
    """Coordinates of a tensor observation grid: axis j holds origin_j + step_j * i,
    i = 0 .. npts_j - 1."""
    return [float(origin[j]) + float(step[j]) * np.arange(int(npts[j]), dtype=np.float64)
            for j in range(len(npts))]


def paper_observation_grid(d: int):
    """The grid of Sec. 4 on which eigenfunctions are compared: [-5a, 5a]^d with
    a = 10^(3-d) and spacing 0.1.  Returns (origin, step, npts) per axis."""
    a = 10.0 ** (3 - d)
    n = int(round(10.0 * a / 0.1)) + 1
    return [-5.0 * a] * d, [0.1] * d, [n] * d


def eigenfunction_on_grid(P, labels: np.ndarray, U: np.ndarray, origin, step, npts) -> np.ndarray:
    """u(xi) = sum_k U_k exp(i (P_paper k) . xi) = sum_k U_k exp(i 2 pi (P k) . xi)
    over the labels k of the coefficient vector U (eq:int, the interpolant
    I_{K,L}; P without the 2 pi), at every point of a tensor grid (shape npts,
    first axis slowest).  The exponential of the sum over the d coordinates is
    taken as the product of the d per-axis exponentials."""
    P = np.asarray(P, dtype=np.float64)
    d = P.shape[0]
    U = np.asarray(U, dtype=np.complex128).ravel()
    f = np.asarray(labels, dtype=np.float64) @ P.T          # N x d: the frequencies P k
    axes = observation_axes(origin, step, npts)
    E = [np.exp(1j * TWO_PI * np.outer(axes[j], f[:, j])) for j in range(d)]   # npts_j x N
    out = np.empty(tuple(int(x) for x in npts), dtype=np.complex128)
    lead = [int(x) for x in npts[:-1]]
    for idx in np.ndindex(*lead) if lead else [()]:
        w = U.copy()
        for j, i in enumerate(idx):
            w = w * E[j][i]
        out[idx] = E[d - 1] @ w
    return out


def normalise_at_max(u: np.ndarray) -> np.ndarray:
    """u divided by its value at the (first) point of largest modulus, which
    fixes the phase and makes the maximal modulus 1 (Sec. 4: eigenfunctions are
    compared after division by their maximal modulus)."""
    flat = np.asarray(u).ravel()
    return np.asarray(u) / flat[int(np.argmax(np.abs(flat)))]


def eigenfunction_error(u: np.ndarray, u_ref: np.ndarray) -> float:
    """E_f = || u - u* ||_inf on the observation grid, both normalised by
    normalise_at_max (Sec. 4)."""
    return float(np.max(np.abs(normalise_at_max(u) - normalise_at_max(u_ref))))
