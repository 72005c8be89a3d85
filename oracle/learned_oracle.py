"""Plain float64 reference of the learned preconditioner.

TEST INFRASTRUCTURE ONLY: used by the tests (and nothing in the product path).
It shares no code with the HIP library.

The paper preconditions its LOBPCG solves with the diagonal M of eq:precond
(Sec. 4.1).  The library adds a trained preconditioner that starts from M and
falls back to it; this module writes that operator out from its definition:

    T(R) = D0 * R + b1 (C E + a)^H E (C E + a) R
         = (D0 + b1 a^2 E) * R + 2 a b1 E * C(E * R) + b1 E * C(E * C(E * R))
    D0 = M * (1 + exp(o0[shell])) / 2,  E = M * exp(o1[shell]),
    a = beta0,  b1 = max(beta1, 0)

where C is the potential block of H~ (H~ minus its kinetic diagonal, i.e. the
wrapped convolution with the Vhat_m, Sec. 4.1) and (o0, o1) = MLP(features of
the kinetic-energy shell).  The MLP has 8 inputs, three hidden layers of 256
with the exact GELU x Phi(x), and 2 linear outputs; its weight matrices are
used after rounding the float32 masters to bfloat16 (nearest, ties to even).

Shells: s(k) = min(S-1, floor(S sqrt(e_k / e_max))), e_k = 1/2 |2 pi P k|^2.
Features of shell s (c = (s+1/2)/S, e = e_max c^2, nu = sum_{m!=0} |Vhat_m|,
v0 = Re Vhat_0, sigma = max(0, nu - v0), S2 = sum_{m!=0} |Vhat_m|^2,
h = e + v0 + sigma; 0/0 read as 0):
    c, log(1+e)/8, e/(e+nu), log(1+nu)/4, h^2/(h^2+S2), nu/h, log(1+e_max)/8,
    sqrt(e)/(sqrt(e)+sqrt(nu)).

Training loss of an iterate block X (N x m) given the exact lowest m
eigenvalues lam: with (Y, theta) the Ritz pairs of span(X), R = H Y - Y theta
and theta' the lowest m Ritz values of span([Y, T(R)]),
    loss = sum_j (theta'_j - lam_j) / sum_j (theta_j - lam_j),
the share of eigenvalue error left after one Rayleigh-Ritz step.

The gradient is derived by hand (the Ritz-value derivative
d theta'_j / dW = 2 (H - theta'_j) y'_j c'_{W,j}^H, then the chain rule through
T, the two convolution layers, the shell reduction and the MLP) and checked
against central finite differences of ``rr_loss`` in the CPU tests.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.special import erf

FEATURES = 8
HIDDEN = 256
DIMS = (FEATURES, HIDDEN, HIDDEN, HIDDEN, 2)


# ---------------------------------------------------------------------------
# parameter vector
# ---------------------------------------------------------------------------

def layout():
    """[(offset_W, shape_W, offset_b, size_b)] for the 4 layers, and the offset of beta."""
    out, off = [], 0
    for l in range(4):
        a, b = DIMS[l], DIMS[l + 1]
        out.append((off, (a, b), off + a * b, b))
        off += a * b + b
    return out, off


def nparams() -> int:
    return layout()[1] + 2


def bf16_round(w) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(np.asarray(w, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params, round_weights: bool = True):
    """(list of (W, b) float64, beta) from the parameter vector."""
    p = np.asarray(params)
    lay, off_beta = layout()
    layers = []
    for ow, shp, ob, nb in lay:
        W = p[ow:ow + shp[0] * shp[1]]
        W = bf16_round(W) if round_weights else np.asarray(W, dtype=np.float64)
        layers.append((W.reshape(shp), np.asarray(p[ob:ob + nb], dtype=np.float64)))
    beta = np.asarray(p[off_beta:off_beta + 2], dtype=np.float64)
    return layers, beta


# ---------------------------------------------------------------------------
# shells and features
# ---------------------------------------------------------------------------

def shell_map(kin, S: int):
    """Shell of each entry, and a mask of entries whose S sqrt(e/e_max) lies
    within 1e-9 of an integer (where rounding alone can move the floor)."""
    kin = np.asarray(kin, dtype=np.float64)
    emax = float(kin.max()) if kin.size else 0.0
    if emax <= 0.0:
        return np.zeros(kin.shape, dtype=np.int64), np.zeros(kin.shape, dtype=bool)
    x = S * np.sqrt(kin / emax)
    s = np.minimum(np.floor(x), S - 1).astype(np.int64)
    frac = np.abs(x - np.round(x))
    amb = (frac < 1e-9) & (np.round(x) > 0) & (np.round(x) < S)
    return s, amb


def potential_scalars(modes, vhat):
    """(nu, v0, S2): sum and sum of squares of |Vhat_m| over m != 0, and Re Vhat_0."""
    modes = np.asarray(modes).reshape(len(vhat), -1) if len(vhat) else np.zeros((0, 1))
    vh = np.asarray(vhat, dtype=np.complex128)
    zero = np.all(modes == 0, axis=1) if len(vh) else np.zeros(0, dtype=bool)
    nu = float(np.abs(vh[~zero]).sum())
    S2 = float((np.abs(vh[~zero]) ** 2).sum())
    v0 = float(vh[zero].real.sum())
    return nu, v0, S2


def shell_features(S: int, emax: float, nu: float, v0: float, S2: float) -> np.ndarray:
    def ratio(a, b):
        return a / b if b > 0 else 0.0
    sigma = max(0.0, nu - v0)
    F = np.zeros((S, FEATURES))
    for s in range(S):
        c = (s + 0.5) / S
        e = emax * c * c
        h = e + v0 + sigma
        F[s] = [c, math.log1p(e) / 8, ratio(e, e + nu), math.log1p(nu) / 4, ratio(h * h, h * h + S2),
                ratio(nu, h), math.log1p(emax) / 8, ratio(math.sqrt(e), math.sqrt(e) + math.sqrt(nu))]
    return F


# ---------------------------------------------------------------------------
# MLP
# ---------------------------------------------------------------------------

def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def mlp_forward(layers, X):
    """O (S x 2) and the cache [(input, pre-activation)] per layer."""
    cache = []
    h = np.asarray(X, dtype=np.float64)
    for l, (W, b) in enumerate(layers):
        z = h @ W + b
        cache.append((h, z))
        h = gelu(z) if l < len(layers) - 1 else z
    return h, cache


def mlp_backward(layers, cache, dO):
    """Gradients [(dW, db)] of sum(dO * O)."""
    grads = [None] * len(layers)
    d = np.asarray(dO, dtype=np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        x, z = cache[l]
        if l < len(layers) - 1:
            d = d * gelu_grad(z)
        grads[l] = (x.T @ d, d.sum(axis=0))
        d = d @ W.T
    return grads


# ---------------------------------------------------------------------------
# the preconditioner, its loss and gradient
# ---------------------------------------------------------------------------

def potential_block(H: sp.spmatrix, kin) -> sp.csr_matrix:
    """C = H~ - diag(kinetic): the wrapped convolution with the Vhat_m (Sec. 4.1)."""
    return (sp.csr_matrix(H) - sp.diags(np.asarray(kin, dtype=np.float64))).tocsr()


def scales(M, shell, O):
    return 0.5 * M * (1.0 + np.exp(O[shell, 0])), M * np.exp(O[shell, 1])


def layer_coefficients(beta):
    """(a, b1) -> coefficients of E A, E Cc and the extra diagonal E in the expanded form."""
    a = float(beta[0])
    b1 = max(float(beta[1]), 0.0)
    return 2.0 * a * b1, b1, b1 * a * a


def precond_apply(C, M, shell, O, beta, R):
    """T(R) column by column (R is N x m); also returns A = C(E R), Cc = C(E A)."""
    D0, E = scales(M, shell, O)
    c0, c1, dl = layer_coefficients(beta)
    R = np.asarray(R, dtype=np.complex128)
    A = C @ (E[:, None] * R)
    Cc = C @ (E[:, None] * A)
    T = (D0 + dl * E)[:, None] * R + E[:, None] * (c0 * A + c1 * Cc)
    return T, A, Cc


def _backprop(layers, cache, beta, C, M, shell, O, R, A, Cc, G):
    """Parameter gradient of a loss whose derivative with respect to T(R) is G."""
    S = O.shape[0]
    D0, E = scales(M, shell, O)
    c0, c1, dl = layer_coefficients(beta)
    # T = (D0 + dl E) R + E (c0 A + c1 Cc), A = C(E R), Cc = C(E A); C Hermitian
    B1 = C @ (E[:, None] * G)
    B2 = C @ (E[:, None] * B1)

    def re(x, y):  # sum over columns of Re(conj(x) y)
        return np.sum((np.conj(x) * y).real, axis=1)

    dD0 = re(G, R)
    dE = c0 * (re(G, A) + re(B1, R)) + c1 * (re(G, Cc) + re(B1, A) + re(B2, R)) + dl * re(G, R)
    g0 = np.sum(re(G, E[:, None] * A))
    g1 = np.sum(re(G, E[:, None] * Cc))
    gd = np.sum(re(G, E[:, None] * R))
    a, b1 = float(beta[0]), max(float(beta[1]), 0.0)
    # beta1 < 0 passes the gradient of its positive side (as the library does)
    dbeta = np.array([2 * b1 * g0 + 2 * a * b1 * gd, 2 * a * g0 + g1 + a * a * gd])
    dO = np.zeros((S, 2))
    np.add.at(dO[:, 0], shell, dD0 * 0.5 * M * np.exp(O[shell, 0]))
    np.add.at(dO[:, 1], shell, dE * E)
    grads = mlp_backward(layers, cache, dO)
    grad = np.zeros(nparams())
    lay, off_beta = layout()
    for (ow, shp, ob, nb), (dW, db) in zip(lay, grads):
        grad[ow:ow + shp[0] * shp[1]] = dW.reshape(-1)
        grad[ob:ob + nb] = db
    grad[off_beta:off_beta + 2] = dbeta
    return grad


def _rr_parts(params, H, C, M, shell, X, Xblk, lam, round_weights):
    layers, beta = unpack(params, round_weights)
    O, cache = mlp_forward(layers, X)
    Xb = np.asarray(Xblk, dtype=np.complex128)
    m = Xb.shape[1]
    HX = H @ Xb
    Am = Xb.conj().T @ HX
    theta, Cm = sla.eigh(0.5 * (Am + Am.conj().T), Xb.conj().T @ Xb)
    Y = Xb @ Cm
    HY = HX @ Cm
    R = HY - Y * theta[None, :]
    W, A, Cc = precond_apply(C, M, shell, O, beta, R)
    S = np.concatenate([Y, W], axis=1)
    HS = np.concatenate([HY, H @ W], axis=1)
    A2 = S.conj().T @ HS
    theta2, C2 = sla.eigh(0.5 * (A2 + A2.conj().T), S.conj().T @ S)
    lam = np.asarray(lam, dtype=np.float64)
    D = float(np.sum(theta[:m] - lam[:m]))
    num = float(np.sum(theta2[:m] - lam[:m]))
    return dict(layers=layers, beta=beta, O=O, cache=cache, R=R, A=A, Cc=Cc, S=S, HS=HS, theta2=theta2, C2=C2,
                D=D, loss=num / D, m=m)


def rr_loss(params, H, C, M, shell, X, Xblk, lam, round_weights: bool = True) -> float:
    return _rr_parts(params, H, C, M, shell, X, Xblk, lam, round_weights)["loss"]


def rr_loss_and_grad(params, H, C, M, shell, X, Xblk, lam, round_weights: bool = True):
    """(loss, gradient over the parameter vector), float64."""
    q = _rr_parts(params, H, C, M, shell, X, Xblk, lam, round_weights)
    m = q["m"]
    C2m = q["C2"][:, :m]
    C2W = q["C2"][m:, :m]
    # d theta'_j / dW = 2 (HS c'_j - theta'_j S c'_j) c'_{W,j}^H, summed and divided by D
    G = (2.0 / q["D"]) * ((q["HS"] @ C2m) - (q["S"] @ (C2m * q["theta2"][None, :m]))) @ C2W.conj().T
    grad = _backprop(q["layers"], q["cache"], q["beta"], C, M, shell, q["O"], q["R"], q["A"], q["Cc"], G)
    return q["loss"], grad


def init_params(seed: int, zero_last: bool = True) -> np.ndarray:
    """A parameter vector in the library's initial form (hidden layers uniform
    in +-1/sqrt(fan_in), last layer and beta zero); numpy's generator, so the
    values differ from the library's own initial draw."""
    rng = np.random.default_rng(seed)
    p = np.zeros(nparams(), dtype=np.float32)
    lay, _ = layout()
    for l, (ow, shp, ob, nb) in enumerate(lay):
        if l == 3 and zero_last:
            continue
        bound = 1.0 / math.sqrt(shp[0])
        p[ow:ow + shp[0] * shp[1]] = rng.uniform(-bound, bound, shp[0] * shp[1])
        p[ob:ob + nb] = rng.uniform(-bound, bound, nb)
    return p
