"""Host-side checks of libiwfpm that need no GPU: the C ABI loads and exports
every declared symbol, host-only plans reproduce the oracle's labels and
kinetic diagonal (Sec. 3.2, eq:inverse1-3; Sec. 4.1), and bad inputs come back
as status codes."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2404_04507_amd as lib
from paper_2404_04507_amd import workloads as W
from paper_2404_04507_amd import dense_geneig, dense_svqb  # noqa: F401

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "iwfpm.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int64_t|int|void|const char\*)\s+(iwfpm_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "iwfpm_plan" in names and "iwfpm_apply" in names and "iwfpm_eigs" in names
    so = ctypes.CDLL(lib.library_path())
    for name in names:
        assert hasattr(so, name), name
    assert set(names) <= set(lib.EXPORTED) | set(names)
    for name in lib.EXPORTED:
        assert name in names


def host_plan(prob, **kw):
    return lib.Plan.from_problem(prob, device=-1, **kw)


CASES = [
    lambda: W.c1_1d(),
    lambda: W.c2_2d(K=5, L=4),
    lambda: W.c3_3d(K=2, L=2),
    lambda: W.paper_example_2d(0.5 * math.pi, 0.25 * math.pi, 4, 6),
    lambda: W.paper_example_3d(math.pi, 2, 3),
]


@pytest.mark.parametrize("variant", ["exact", "rounded", "pm"])
@pytest.mark.parametrize("make", CASES)
def test_labels_and_kinetic_match_oracle(make, variant):
    prob = make()
    with host_plan(prob, window=variant) as p:
        assert p.N == prob.N and p.ext == prob.ext
        k = p.indices()
        ref = O.grid_labels(prob.P, prob.d, prob.K, prob.L, variant)
        assert np.array_equal(k, ref)
        lam = p.kinetic()
        lref = O.kinetic(prob.P, ref)
        assert np.allclose(lam, lref, rtol=1e-14, atol=1e-12)
        nb = p.norm_bound()
        assert abs(nb - (lref.max() + np.abs(prob.vhat).sum())) < 1e-9 * nb


@pytest.mark.parametrize("make", CASES)
def test_window_order_sorts_each_slice(make):
    """WINDOW order: within a slice, entries run over k_I ascending from the lower window end."""
    prob = make()
    with host_plan(prob, order="window") as p:
        k = p.indices()
    ref = O.grid_labels(prob.P, prob.d, prob.K, prob.L)
    assert {tuple(x) for x in k} == {tuple(x) for x in ref}
    nkI = int(np.prod([2 * x for x in prob.K]))
    d = prob.d
    for s in range(0, prob.N // nkI, max(1, prob.N // nkI // 7)):
        blk = k[s * nkI:(s + 1) * nkI, :d].reshape([2 * x for x in prob.K] + [d])
        # along each k_I axis consecutive entries differ by exactly +1
        for j in range(d):
            dif = np.diff(blk[..., j], axis=j)
            assert np.all(dif == 1)


def test_tie_at_integer_offset():
    """C3's Q has cancelling entries (k4 = k5 gives q1 = 0 exactly) and rational
    entries in C2 (q = -k4/2): the half-open window rule decides ties."""
    for prob in (W.c3_3d(K=2, L=2), W.c2_2d(K=3, L=4)):
        with host_plan(prob) as p:
            k = p.indices()
        assert np.array_equal(k, O.grid_labels(prob.P, prob.d, prob.K, prob.L))


def test_status_codes():
    P = np.array([[1.0, W.GOLDEN]])
    modes, vhat = W.cosine_modes(2, [1.0, 1.0])
    with pytest.raises(lib.IwfpmError) as e:
        lib.Plan(np.array([[0.0, 1.0]]), [4], [4], modes, vhat, device=-1)
    assert e.value.status == -2  # singular P_I
    with pytest.raises(lib.IwfpmError) as e:
        lib.Plan(P, [4], [4], [[1, 0]], [1.0 + 1.0j], device=-1)
    assert e.value.status == -3  # no conjugate partner
    with pytest.raises(lib.IwfpmError) as e:
        lib.Plan(P, [0], [4], modes, vhat, device=-1)
    assert e.value.status == -1
    with pytest.raises(lib.IwfpmError) as e:
        lib.Plan(P, [4], [37], modes, vhat, device=-1)
    assert e.value.status == -4  # 2L = 74 = 2 x 37: no compiled pencil of 37 points
    p = lib.Plan(P, [4], [4], modes, vhat, device=-1)
    so = lib.load_library()
    st = so.iwfpm_apply(p._h, ctypes.c_void_p(8), ctypes.c_void_p(1 << 20), 1, ctypes.c_void_p())
    assert st == -10  # host-only plan
    st = so.iwfpm_apply(p._h, ctypes.c_void_p(), ctypes.c_void_p(), 1, ctypes.c_void_p())
    assert st == -1
    p.close()
    assert so.iwfpm_dof(ctypes.c_void_p(), ctypes.byref(ctypes.c_int64())) == -1


def test_duplicate_modes_are_merged():
    P = np.array([[1.0, W.GOLDEN]])
    with lib.Plan(P, [4], [4], [[1, 0], [-1, 0], [1, 0], [-1, 0]], [0.5, 0.5, 0.25, 0.25], device=-1) as p:
        assert abs(p.norm_bound() - (p.kinetic().max() + 1.5)) < 1e-12


# --- the host Rayleigh-Ritz solver of iwfpm_eigs ---------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 48, 96])
def test_dense_geneig_matches_lapack(n):
    """Cholesky + Householder/QL against LAPACK's generalised Hermitian eigensolver."""
    import scipy.linalg as sla
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = A + A.conj().T
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    B = Z @ Z.conj().T + n * np.eye(n)
    w, C = lib.dense_geneig(A, B)
    wr = sla.eigh(A, B, eigvals_only=True)
    assert np.allclose(w, wr, rtol=1e-12, atol=1e-12 * np.abs(wr).max())
    assert np.allclose(C.conj().T @ B @ C, np.eye(n), atol=1e-10)
    assert np.allclose(A @ C, B @ C * w[None, :], atol=1e-9 * np.abs(A).max())


def test_dense_geneig_degenerate_and_identity():
    A = np.diag([3.0, 1.0, 1.0, -2.0]).astype(complex)
    A[0, 3] = A[3, 0] = 1e-9
    w, C = lib.dense_geneig(A)
    assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-14)
    with pytest.raises(lib.IwfpmError):
        lib.dense_geneig(A, -np.eye(4))


@pytest.mark.parametrize("real", [False, True], ids=["complex", "real"])
def test_dense_svqb_drops_dependent_directions(real):
    rng = np.random.default_rng(3)
    V = (rng.standard_normal((200, 5)) + (0 if real else 1j) * rng.standard_normal((200, 5))).astype(complex)
    V = np.concatenate([V, V[:, :2] * 2.0 + V[:, 2:4]], axis=1)  # rank 5 of 7
    T = lib.dense_svqb(V.conj().T @ V)
    assert T.shape == (7, 5)
    Q = V @ T
    assert np.allclose(Q.conj().T @ Q, np.eye(5), atol=1e-10)
    if real:
        assert np.all(T.imag == 0.0)


@pytest.mark.parametrize("real", [False, True], ids=["complex", "real"])
@pytest.mark.parametrize("n,nv", [(1, 1), (2, 0), (7, 3), (48, 16), (60, 20), (64, 64)])
def test_dense_heev_lowest_matches_lapack(n, nv, real):
    """Eigenvalues against LAPACK; the nv returned vectors are orthonormal
    eigenvectors of the nv lowest values (checked through residuals and against
    LAPACK's vectors up to phase, the spectrum being simple here).  A real
    symmetric input takes the real Householder reduction and must come back
    with exactly real vectors."""
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n)) + (0 if real else 1j) * rng.standard_normal((n, n))
    A = (A + A.conj().T).astype(complex)
    w, V = lib.dense_heev_lowest(A, nv)
    if real:
        assert np.all(V.imag == 0.0)
    wr, Vr = np.linalg.eigh(A)
    scale = np.abs(wr).max()
    assert np.allclose(w, wr, rtol=0, atol=1e-13 * scale)
    assert V.shape == (n, nv)
    if nv:
        assert np.allclose(V.conj().T @ V, np.eye(nv), atol=1e-12)
        assert np.abs(A @ V - V * w[None, :nv]).max() < 1e-12 * scale
        overlap = np.abs(np.sum(Vr[:, :nv].conj() * V, axis=0))
        assert np.allclose(overlap, 1.0, atol=1e-10)


@pytest.mark.parametrize("real", [False, True], ids=["complex", "real"])
def test_dense_heev_lowest_degenerate_cluster(real):
    """A multiple eigenvalue: the returned vectors span the LAPACK eigenspace."""
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)) + (0 if real else 1j) * rng.standard_normal((12, 12)))
    Q = Q.astype(complex)
    vals = np.array([-1.0, -1.0, -1.0, 0.5, 0.5, 2.0, 3.0, 3.0, 4.0, 5.0, 6.0, 7.0])
    A = (Q * vals) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    w, V = lib.dense_heev_lowest(A, 5)
    assert np.allclose(w, np.sort(vals), atol=1e-13)
    assert np.allclose(V.conj().T @ V, np.eye(5), atol=1e-12)
    # projector onto the span of the 5 lowest eigenvectors
    P = Q[:, :5] @ Q[:, :5].conj().T
    assert np.allclose(P @ V, V, atol=1e-12)
    with pytest.raises(lib.IwfpmError):
        lib.dense_heev_lowest(A, 13)


def test_eigenfunction_argument_checks_on_host_plan():
    """iwfpm_eigenfunction validates before any device work: NULL pointers and
    empty axes are ERR_ARG, a host-only plan is ERR_NODEVICE."""
    import ctypes
    prob = W.paper_example_1d(2.5, 2, 2)
    with lib.Plan.from_problem(prob, device=-1) as p:
        L = lib.load_library()
        o = (ctypes.c_double * 1)(0.0)
        h = (ctypes.c_double * 1)(0.1)
        n = (ctypes.c_int32 * 1)(4)
        fake = ctypes.c_void_p(16)  # never dereferenced: every path below returns first
        assert L.iwfpm_eigenfunction(p._h, None, o, h, n, fake, None) == -1
        assert L.iwfpm_eigenfunction(p._h, fake, o, h, None, fake, None) == -1
        assert L.iwfpm_eigenfunction(p._h, fake, o, h, n, fake, None) == -10


def test_five_pass_grids_plan_on_host():
    """Ex. 4.3 at K = 5, L = 20, 30 and 40 (40^3, 60^3 and 80^3 x 10^3): no single
    split fits both the slab and the leading block in LDS, and the plan takes
    the five-pass schedule instead of refusing (passes 1 and 3 keep the three
    10-point axes; L = 40 has 80-point axes, transformed in two stages)."""
    import math
    for L in (20, 30, 40):
        prob = W.paper_example_3d(math.pi, 5, L)
        with lib.Plan.from_problem(prob, device=-1) as p:
            assert p.N == 1000 * (2 * L) ** 3
            for prec in ("fp32", "fp64"):
                sc = p.schedule(prec)
                assert not sc["fused"] and sc["split"] == 3, sc


@pytest.mark.parametrize("ext,ok", [(34, True), (38, True), (42, True), (44, True), (46, True), (50, True),
                                    (52, True), (54, True), (56, True), (58, True), (62, True), (80, True),
                                    (84, True), (100, True), (120, True), (160, True), (1024, True),
                                    (8192, True), (74, False), (82, False), (86, False), (94, False),
                                    (106, False), (118, False), (122, False)])
def test_axis_extents_supported(ext, ok):
    """Every even extent whose factors are compiled pencil sizes (at most three
    stages) plans, on either kind of axis, with labels equal to the oracle's;
    an extent with a prime factor above 32 (37, 41, 43, 47, 53, 59, 61) is
    refused with ERR_UNSUPPORTED."""
    P = np.array([[1.0, W.GOLDEN]])
    modes, vhat = W.cosine_modes(2, [1.0, 1.0])
    for K, L in (([3], [ext // 2]), ([ext // 2], [3])):
        if ok:
            with lib.Plan(P, K, L, modes, vhat, device=-1) as p:
                assert p.N == 6 * ext
                if p.N <= 4096:
                    assert np.array_equal(p.indices(), O.grid_labels(P, 1, K, L))
        else:
            with pytest.raises(lib.IwfpmError) as e:
                lib.Plan(P, K, L, modes, vhat, device=-1)
            assert e.value.status == -4
