"""Seeded synthetic inputs: projection matrices, windows, potential modes and
random vectors for the quasiperiodic Schroedinger workloads.

This module only *describes* problems (it holds none of the method's
arithmetic), so both the HIP library's tests/benchmark and the CPU oracle may
draw their inputs from it.

P follows the library convention: the kinetic energy of mode k is
1/2 |2 pi P k|^2.  The paper's examples (Sec. 4) write P with the 2 pi (and
beta) inside; ``paper_example_*`` divide it out.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED = 2404045070
GOLDEN = (math.sqrt(5.0) - 1.0) / 2.0  # alpha of Ex. 4.1 and Ex. 4.3


@dataclass
class Problem:
    """One IWFPM eigenproblem instance."""
    name: str
    d: int
    P: np.ndarray            # d x n, float64
    K: list                  # length d
    L: list                  # length n - d
    modes: np.ndarray        # n_modes x n, int
    vhat: np.ndarray         # n_modes, complex128
    nev: int = 8
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.P.shape[1]

    @property
    def ext(self) -> tuple:
        return tuple(2 * x for x in self.L) + tuple(2 * x for x in self.K)

    @property
    def N(self) -> int:
        return int(np.prod(self.ext))


def cosine_modes(n: int, weights, const: float = 0.0):
    """Modes of const + sum_j w_j cos(y_j): Vhat_{+-e_j} = w_j / 2."""
    modes, vhat = [], []
    if const != 0.0:
        modes.append([0] * n)
        vhat.append(const)
    for j, w in enumerate(weights):
        if w == 0.0:
            continue
        for s in (1, -1):
            e = [0] * n
            e[j] = s
            modes.append(e)
            vhat.append(w / 2.0)
    return np.array(modes, dtype=np.int64).reshape(-1, n), np.array(vhat, dtype=np.complex128)


# --- the five benchmark workloads ------------------------------------------

def c1_1d(lam: float = 1.0, K: int = 8, L: int = 16) -> Problem:
    """1D QSE lifted to a 2D torus: P = [1, alpha], V = lam (cos y1 + cos y2)."""
    P = np.array([[1.0, GOLDEN]])
    modes, vhat = cosine_modes(2, [lam, lam])
    return Problem("1d_lifted_2d", 1, P, [K], [L], modes, vhat, nev=8,
                   meta={"lam": lam})


def rot_pair_P(angle: float = math.pi / 6.0) -> np.ndarray:
    """Two square lattices, the second rotated by ``angle``: P = [I | R(angle)]."""
    c, s = math.cos(angle), math.sin(angle)
    return np.array([[1.0, 0.0, c, -s],
                     [0.0, 1.0, s, c]])


def c2_2d(lam: float = 0.5, K: int = 12, L: int = 16) -> Problem:
    """2D QSE lifted to 4D: rotated square-lattice pair, V = lam sum_j cos y_j."""
    P = rot_pair_P()
    modes, vhat = cosine_modes(4, [lam] * 4)
    return Problem("2d_lifted_4d", 2, P, [K, K], [L, L], modes, vhat, nev=16,
                   meta={"lam": lam})


def cubic_pair_P() -> np.ndarray:
    """Cubic lattice plus a copy rotated by pi/4 in the x1x2 plane, x3 scaled by sqrt2-1."""
    c = math.sqrt(2.0) / 2.0
    Q = np.array([[c, -c, 0.0],
                  [c, c, 0.0],
                  [0.0, 0.0, math.sqrt(2.0) - 1.0]])
    return np.concatenate([np.eye(3), Q], axis=1)


def c3_3d(lam: float = 3.0, K: int = 8, L: int = 8) -> Problem:
    """3D QSE lifted to 6D, V = lam sum_j cos y_j."""
    P = cubic_pair_P()
    modes, vhat = cosine_modes(6, [lam] * 6)
    return Problem("3d_lifted_6d", 3, P, [K] * 3, [L] * 3, modes, vhat, nev=16,
                   meta={"lam": lam})


def c4_sweep(count: int = 64, L: int = 16, seed: int = SEED) -> list:
    """Batched coupling sweep: lam ~ U[0.1, 10], K ~ U{6..14}, the 2D/4D geometry."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed + i)
        lam = float(rng.uniform(0.1, 10.0))
        K = int(rng.integers(6, 15))
        p = c2_2d(lam=lam, K=K, L=L)
        p.name = f"sweep_{i}"
        p.nev = 8
        p.meta["seed"] = seed + i
        out.append(p)
    return out


def c5_heldout_lams(count: int = 32, seed: int = SEED) -> list:
    """Held-out couplings lam_j = 0.1 + 9.9 (j + U(0.25, 0.75)) / count."""
    rng = np.random.default_rng(seed + 1000)
    return [0.1 + 9.9 * (j + float(rng.uniform(0.25, 0.75))) / count for j in range(count)]


# --- the paper's own examples (Sec. 4) --------------------------------------

def paper_example_1d(v0: float, K: int, L: int) -> Problem:
    """Ex. 4.1: v = v0 [2 - cos 2pi x - cos 2pi alpha x], P_paper = 2pi (1, alpha)."""
    P = np.array([[1.0, GOLDEN]])
    modes, vhat = cosine_modes(2, [-v0, -v0], const=2.0 * v0)
    return Problem("paper_ex1", 1, P, [K], [L], modes, vhat, nev=1, meta={"v0": v0})


def paper_example_2d(beta: float, theta: float, K: int, L: int) -> Problem:
    """Ex. 4.2: v = 4 - [cos b x1 + 2 cos b x2 + cos(b x1 cos t + b x2 sin t)]."""
    P = (beta / (2.0 * math.pi)) * np.array([[1.0, 0.0, math.cos(theta)],
                                             [0.0, 1.0, math.sin(theta)]])
    modes, vhat = cosine_modes(3, [-1.0, -2.0, -1.0], const=4.0)
    return Problem("paper_ex2", 2, P, [K, K], [L], modes, vhat, nev=1,
                   meta={"beta": beta, "theta": theta})


def paper_example_3d(beta: float, K: int, L: int, theta: float = 0.2 * math.pi) -> Problem:
    """Ex. 4.3: v = 6 - sum of six cosines, P (3 x 6) with a theta rotation and alpha."""
    c, s = math.cos(theta), math.sin(theta)
    P = (beta / (2.0 * math.pi)) * np.array([[1.0, 0.0, 0.0, c, -s, 0.0],
                                             [0.0, 1.0, 0.0, s, c, 0.0],
                                             [0.0, 0.0, 1.0, 0.0, 0.0, GOLDEN]])
    modes, vhat = cosine_modes(6, [-1.0] * 6, const=6.0)
    return Problem("paper_ex3", 3, P, [K] * 3, [L] * 3, modes, vhat, nev=1,
                   meta={"beta": beta})


def fig1_window(K: int = 2, L: int = 6) -> Problem:
    """Fig. 1: d=1, n=2, P = (1, (sqrt5+1)/2), K=2, L=6 (no potential)."""
    P = np.array([[1.0, (math.sqrt(5.0) + 1.0) / 2.0]])
    return Problem("fig1", 1, P, [K], [L], np.zeros((0, 2), dtype=np.int64),
                   np.zeros(0, dtype=np.complex128), nev=1)


# --- seeded random blocks ---------------------------------------------------

def random_block(N: int, m: int, seed: int = SEED) -> np.ndarray:
    """Complex standard-normal N x m block (column-major use: column j is vector j)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m))
    return X / math.sqrt(2.0)
