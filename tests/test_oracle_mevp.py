"""Pins of the oracle's invert-Krylov MEVP (Algorithm 1) and of its small
Hessenberg exponential, against closed forms, dense linear algebra and the
paper's own residual identity."""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg as spla

import netgen
from oracle import InvertKrylov, hessenberg_phi
from tests.exact import expm_hJ


def test_phi_scalar_closed_form():
    # m = 1, H = [mu]: M = h/mu, d = 1 - exp(h/mu), rho = beta*h21*|exp(h/mu)/mu|
    for mu, h in [(-1e-12, 1e-13), (-3e-11, 2e-12), (-1e-15, 1e-12)]:
        d, rho = hessenberg_phi(np.array([[mu]]), 0.7, 2.0, h)
        e = np.exp(h / mu)
        assert d[0] == pytest.approx(1 - e, rel=1e-14, abs=1e-300)
        assert rho == pytest.approx(2.0 * 0.7 * abs(e / mu), rel=1e-13, abs=1e-300)


def test_phi_two_by_two_closed_form():
    # H with real distinct eigenvalues: e^{hH^{-1}} e1 through its eigenvectors
    H = np.array([[-2e-12, 0.5e-12], [1e-12, -5e-12]])
    h = 3e-12
    lam, W = np.linalg.eig(H)
    M_eig = h / lam
    y = (W * np.exp(M_eig)) @ np.linalg.solve(W, [1.0, 0.0])
    d, rho = hessenberg_phi(H, 0.3, 1.5, h)
    assert np.allclose(d, np.array([1.0, 0.0]) - y, rtol=1e-12, atol=1e-15)
    Hinv_y = np.linalg.solve(H, y)
    assert rho == pytest.approx(1.5 * 0.3 * abs(Hinv_y[1]), rel=1e-12)


def test_phi_small_argument_has_no_cancellation():
    # d = (I - e^M) e1 for a slow mode: 1 - exp(-1e-9) must keep full relative accuracy
    d, _ = hessenberg_phi(np.array([[-1.0]]), 0.0, 1.0, 1e-9)
    assert d[0] == pytest.approx(-np.expm1(-1e-9), rel=1e-13)


def _mesh_operator(seed=11, side=8):
    net = netgen.rc_mesh(seed=seed, side=side, T=1e-9, n_loads=4)
    lu = spla.splu(net.G.tocsc())
    C = net.C.tocsr()
    return net, (lambda q: -lu.solve(C @ q))


def test_arnoldi_relation_and_orthogonality():
    net, A = _mesh_operator()
    rng = np.random.default_rng(2)
    v = A(rng.standard_normal(net.n))
    k = InvertKrylov(A, v, 60)
    for _ in range(20):
        k.iterate()
    m = k.m
    V = k.V[:, : m + 1]
    AV = np.column_stack([A(k.V[:, j]) for j in range(m)])
    assert np.linalg.norm(AV - V @ k.H[: m + 1, :m]) <= 1e-11 * np.linalg.norm(AV)
    assert np.linalg.norm(V.T @ V - np.eye(m + 1)) < 1e-10
    # upper Hessenberg
    assert np.all(np.tril(k.H[: m + 1, :m], -2) == 0)


def test_residual_identity_of_the_paper():
    # r_m(h) = C (x_m' - J x_m) = -beta h_{m+1,m} G v_{m+1} e_m^T H_m^{-1} e^{h H_m^{-1}} e1
    net, A = _mesh_operator()
    G = net.G.toarray(); C = net.C.toarray()
    rng = np.random.default_rng(3)
    v = A(rng.standard_normal(net.n))
    k = InvertKrylov(A, v, 60)
    for _ in range(8):
        k.iterate()
    m, beta = k.m, k.beta
    Hm = k.H[:m, :m]; Hinv = np.linalg.inv(Hm)
    h = 2e-13
    import scipy.linalg as sl
    E = sl.expm(h * Hinv)[:, 0]
    Vm = k.V[:, :m]
    lhs = beta * (C @ (Vm @ (Hinv @ E)) + G @ (Vm @ E))
    rhs = -beta * k.H[m, m - 1] * (G @ k.V[:, m]) * (Hinv @ E)[m - 1]
    terms = beta * (np.linalg.norm(C @ (Vm @ (Hinv @ E))) + np.linalg.norm(G @ (Vm @ E)))
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * terms
    # and rho_m is the 2-norm of G^{-1} r_m
    _, rho = k.phi(h)
    assert rho == pytest.approx(np.linalg.norm(np.linalg.solve(G, rhs)), rel=1e-9)


def test_residual_estimate_tracks_true_error():
    net, A = _mesh_operator()
    G = net.G.toarray(); C = net.C.toarray()
    rng = np.random.default_rng(5)
    ratios = []
    for trial in range(3):
        v = A(rng.standard_normal(net.n))
        v /= np.linalg.norm(v)
        for h in (3e-14, 1e-13, 1e-12):
            exact = expm_hJ(G, C, h, v)
            k = InvertKrylov(A, v, 60)
            for _ in range(25):
                k.iterate()
                d, rho = k.phi(h)
                err = np.linalg.norm((v - k.combine(d)) - exact)
                if err > 1e-11:
                    ratios.append(rho / err)
    # rho_m is an estimate of the error (not a bound): within a decade or two
    # on every iterate (it dips when e_m^T H^-1 y passes near zero)
    # and close to it in the median; a dropped factor or a
    # wrong index would shift it by many orders of magnitude
    ratios = np.array(ratios)
    assert ratios.size > 30
    assert np.all(ratios > 1e-3) and np.all(ratios < 20)
    assert 0.3 < np.median(ratios) < 3


def test_exact_when_krylov_space_is_complete():
    # 8-node circuit: after at most rank(C) steps the basis is invariant and the
    # MEVP equals the dense e^{hJ} v
    net = netgen.tiny_linear(3)
    lu = spla.splu(net.G.tocsc())
    A = lambda q: -lu.solve(net.C @ q)
    G = net.G.toarray(); C = net.C.toarray()
    rng = np.random.default_rng(0)
    v = A(rng.standard_normal(net.n))
    h = 5e-12
    k = InvertKrylov(A, v, 60)
    d, rho = k.converge(h, 1e-30)
    assert k.m <= np.linalg.matrix_rank(C)
    assert np.allclose(v - k.combine(d), expm_hJ(G, C, h, v), rtol=1e-10, atol=1e-13 * np.abs(v).max())


def test_zero_vector_is_trivial():
    net, A = _mesh_operator()
    k = InvertKrylov(A, np.zeros(net.n), 10)
    d, rho = k.converge(1e-12, 1e-9)
    assert rho == 0.0 and np.all(k.combine(d) == 0)


def _phi2_scalar(z):
    return (np.exp(z) - 1.0 - z) / z ** 2


def test_phi2_scalar_closed_form():
    # one node: J = -g/c, h phi_2(hJ) C^{-1} b = (h b / c) phi_2(-h g / c)
    from oracle.mevp import InvertKrylov
    g, c, b = 2.0e-3, 5e-15, 1.3e-4
    A = lambda q: -(c * q) / g
    for h in (1e-13, 2.5e-12, 1e-11):
        k = InvertKrylov(A, np.array([b / g]), 4)
        k.iterate()
        got = k.combine(k.phi2(h))[0]
        ref = h * b / c * _phi2_scalar(-h * g / c)
        assert got == pytest.approx(ref, rel=1e-12)


def test_phi2_matches_dense_exponential_on_a_complete_space():
    # h phi_2(hJ) C^{-1} b from the dense augmented exponential, J = -C^{-1} G
    from oracle.mevp import InvertKrylov
    rng = np.random.default_rng(11)
    n = 7
    G = rng.uniform(-1, 1, (n, n)) * 1e-3 + np.eye(n) * 5e-3
    Q = rng.standard_normal((n, n))
    C = (Q @ Q.T + n * np.eye(n)) * 1e-15
    b = rng.standard_normal(n) * 1e-4
    J = -np.linalg.solve(C, G)
    A = lambda q: -np.linalg.solve(G, C @ q)
    for h in (1e-14, 1e-12, 3e-11):
        aug = np.zeros((n + 2, n + 2))
        aug[:n, :n] = h * J
        aug[:n, n] = np.linalg.solve(C, b)
        aug[n, n + 1] = 1.0
        ref = h * scipy.linalg.expm(aug)[:n, n + 1]
        k = InvertKrylov(A, np.linalg.solve(G, b), n)
        for _ in range(n):
            if not k.exact:
                k.iterate()
        got = k.combine(k.phi2(h))
        assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))
