"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Every test here checks the oracle against something other than itself: closed forms,
identities between independently computed matrices, a different algorithm (Lagrange), numpy's
own routines, finite differences, or inequalities the optimisation must satisfy.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bopt, direct, grad, kb, lagrange, nfft


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


# ------------------------------------------------------------------ window (Remark 2.1 reading)

def test_i0_series_matches_numpy():
    z = np.linspace(0.0, 60.0, 241)
    assert np.max(np.abs(kb.i0_series(z) / np.i0(z) - 1)) < 1e-14


def test_window_closed_form_values():
    m, b = 6, kb.shape_b(2.0)
    assert kb.window(np.array([0.0]), m, b)[0] == pytest.approx(np.sinh(b * m) / (np.pi * m), rel=1e-15)
    # edge of the closed support: the limit b/pi; beyond it zero
    assert kb.window(np.array([m, -m]), m, b) == pytest.approx([b / np.pi, b / np.pi], rel=1e-15)
    assert np.all(kb.window(np.array([m + 1e-12, -m - 0.5, 7.0]), m, b) == 0)
    v = np.linspace(-m, m, 101)
    assert np.allclose(kb.window(v, m, b), kb.window(-v, m, b), rtol=0, atol=0)


def test_window_derivative_matches_central_differences():
    m, b = 4, kb.shape_b(2.0)
    v = np.linspace(-m + 0.01, m - 0.01, 77)
    h = 1e-6
    fd = (kb.window(v + h, m, b) - kb.window(v - h, m, b)) / (2 * h)
    an = kb.window_deriv(v, m, b)
    assert np.max(np.abs(fd - an)) / np.max(np.abs(an)) < 1e-8
    # near the edge the small-argument series takes over; check continuity across it
    ve = m - np.array([1e-9, 1e-7, 1e-5, 1e-4])
    fd = (kb.window(ve + 1e-11, m, b) - kb.window(ve - 1e-11, m, b)) / 2e-11
    assert np.allclose(kb.window_deriv(ve, m, b), fd, rtol=1e-3)


# ------------------------------------------------------------------ direct sums (1.1)-(1.3)

@pytest.mark.parametrize("N,M", [(16, 16), (32, 8), (8, 32), (24, 48)])
def test_equispaced_exact_inverse(N, M):
    """Section 3.2: A^*A = N I_M for M <= N and A A^* = M I_N for M >= N, N | M."""
    x = W.equispaced_nodes(N)
    A = direct.ndft_matrix(x, (M,))
    if M <= N:
        assert np.max(np.abs(A.conj().T @ A - N * np.eye(M))) < 1e-12 * N
    if M >= N and M % N == 0:
        assert np.max(np.abs(A @ A.conj().T - M * np.eye(N))) < 1e-12 * M


def test_direct_sum_functions_match_dense_matrix_1d_2d():
    g = W.rng(3)
    for d, M in ((1, (12,)), (2, (6, 8))):
        x = W.uniform_nodes(g, 17, d)
        fh = W.complex_normal(g, (2,) + M)
        A = direct.ndft_matrix(x, M)
        f = direct.ndft(x, fh)
        assert rel(f, fh.reshape(2, -1) @ A.T) < 1e-14
        fr = W.complex_normal(g, (2, 17))
        h = direct.ndft_adjoint(x, fr, M)
        assert rel(h.reshape(2, -1), fr @ A.conj()) < 1e-14


@pytest.mark.parametrize("N", [8, 12, 32, 64])
def test_lagrange_formula_pins_direct_sums(N):
    """(3.5) with (3.4) evaluated directly reproduces f(x_l) of the direct sum, and
    Algorithm 3.3 step 6 returns the coefficients (jittered nodes (3.8))."""
    g = W.rng(N)
    y = W.jittered_nodes_paper(g, N)[:, 0]
    fh = W.complex_normal(g, (N,))
    f = direct.ndft(y[:, None], fh)
    xl = lagrange.aux_nodes(N)
    gl = lagrange.lagrange_values(y, f, xl)
    assert rel(gl, direct.ndft(xl[:, None], fh)) < 1e-12
    assert rel(lagrange.inverse(y, f), fh) < 1e-12


def test_dense_pseudoinverse_recovers_coefficients():
    g = W.rng(5)
    x = W.jittered_nodes(g, 64)
    fh = W.complex_normal(g, (24,))
    A = direct.ndft_matrix(x, (24,))
    f = direct.ndft(x, fh)
    assert rel(np.linalg.pinv(A) @ f, fh) < 1e-12 * np.linalg.cond(A)


def test_exact_phase_reduction_large_k():
    """The split-product phase keeps full accuracy where a naive k*x loses digits."""
    x = np.array([0.123456789012345, -0.4999999999, 0.3333333333333333])
    k = np.array([2 ** 15 - 1, -(2 ** 15)], dtype=np.int64)
    E = direct.phase_matrix(x, k)
    from fractions import Fraction
    for i, xv in enumerate(x):
        for c, kv in enumerate(k):
            fr = Fraction(xv) * kv
            fr = fr - (fr.numerator // fr.denominator)
            ref = np.exp(2j * np.pi * float(fr))
            assert abs(E[i, c] - ref) < 4e-16


# ------------------------------------------------------------------ NFFT (Section 2)

@pytest.mark.parametrize("d,M,N", [(1, (16,), 23), (2, (6, 8), 19)])
def test_nfft_equals_dense_factor_product(d, M, N):
    """trafo == B F D fhat and adjoint == D^* F^* B^* f with the factors built entry by entry
    from (2.4)-(2.6)."""
    g = W.rng(11)
    p = nfft.Params(M, 2.0, 2)
    x = W.uniform_nodes(g, N, d)
    fh = W.complex_normal(g, M)
    B, F, D = nfft.dense_B(x, p), nfft.dense_F(p), nfft.dense_D(p)
    assert rel(nfft.trafo(x, fh, p), B @ F @ D @ fh.ravel()) < 1e-13
    f = W.complex_normal(g, (N,))
    h = nfft.adjoint(x, f, p)
    assert rel(h.ravel(), D.conj().T @ F.conj().T @ B.T @ f) < 1e-13


@pytest.mark.parametrize("d", [1, 2])
def test_nfft_adjointness(d):
    g = W.rng(12)
    M = (32,) if d == 1 else (12, 16)
    p = nfft.Params(M, 2.0, 4)
    x = W.uniform_nodes(g, 200, d)
    fh = W.complex_normal(g, M)
    f = W.complex_normal(g, (200,))
    lhs = np.vdot(f, nfft.trafo(x, fh, p))
    rhs = np.vdot(nfft.adjoint(x, f, p), fh)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def envelope(m, sigma):
    """Window-error envelope for the Kaiser-Bessel NFFT in the form usually quoted in the NFFT
    literature (d = 1): 4 pi (sqrt(m) + m) (1 - 1/sigma)^(1/4) exp(-2 pi m sqrt(1 - 1/sigma))."""
    return 4 * np.pi * (np.sqrt(m) + m) * (1 - 1 / sigma) ** 0.25 * np.exp(-2 * np.pi * m * np.sqrt(1 - 1 / sigma))


def test_nfft_error_envelope_and_rate_1d():
    g = W.rng(13)
    M, N, sigma = 256, 512, 2.0
    x = W.uniform_nodes(g, N, 1)
    fh = W.complex_normal(g, (M,))
    f0 = direct.ndft(x, fh)
    errs = []
    for m in range(2, 8):
        p = nfft.Params((M,), sigma, m)
        e = np.max(np.abs(nfft.trafo(x, fh, p) - f0)) / np.sum(np.abs(fh))
        assert e <= envelope(m, sigma)
        errs.append(e)
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    rate = np.exp(2 * np.pi * np.sqrt(1 - 1 / sigma))   # ~ 85 per unit m at sigma = 2
    assert np.all(ratios > rate / 4) and np.all(ratios < rate * 4)


def test_nfft_error_envelope_2d_and_adjoint():
    g = W.rng(14)
    M = (24, 32)
    x = W.uniform_nodes(g, 300, 2)
    fh = W.complex_normal(g, M)
    f = W.complex_normal(g, (300,))
    for m in (3, 5):
        p = nfft.Params(M, 2.0, m)
        e = np.max(np.abs(nfft.trafo(x, fh, p) - direct.ndft(x, fh))) / np.sum(np.abs(fh))
        assert e <= 2 * envelope(m, 2.0)
        h = nfft.adjoint(x, f, p)
        e2 = np.max(np.abs(h - direct.ndft_adjoint(x, f, M))) / np.sum(np.abs(f))
        assert e2 <= 2 * envelope(m, 2.0)


def test_equispaced_adjoint_of_trafo_is_identity_within_envelope():
    """(1/N) A^* A = I for equispaced nodes, M = N (Section 3.2), through the NFFT pair."""
    N = 64
    x = W.equispaced_nodes(N)
    fh = W.complex_normal(W.rng(15), (N,))
    p = nfft.Params((N,), 2.0, 6)
    back = nfft.adjoint(x, nfft.trafo(x, fh, p), p) / N
    assert np.max(np.abs(back - fh)) < 4 * envelope(6, 2.0) * np.sum(np.abs(fh))


# ------------------------------------------------------------------ B_opt (Algorithm 3.17)

def _dense_K(x, p):
    """K = A D^* F^* (3.14) as a product of the dense factors."""
    A = direct.ndft_matrix(x, p.M)
    return A @ nfft.dense_D(p).conj().T @ nfft.dense_F(p).conj().T


@pytest.mark.parametrize("d,M", [(1, (10,)), (2, (4, 6))])
def test_kernel_formula_matches_dense_product_and_frame_identities(d, M):
    """(3.15): K(x_j - l/M_sigma) equals (A D^* F^*)[j, l]; hence Phi_l2 of (4.6) satisfies
    Phi B^* = (B K^*)^T and B^* Phi = (K^* B)^T (Section 4.2.2)."""
    g = W.rng(21)
    p = nfft.Params(M, 2.0, 1 if d == 2 else 2)
    x = W.uniform_nodes(g, 9, d)
    Kd = _dense_K(x, p)
    S = bopt._grid_points(p)
    xw, _, _ = nfft.prepare_nodes(x, p)
    Kf = np.stack([bopt.kernel_K(xw[j][None, :] - S, p) for j in range(x.shape[0])])
    assert rel(Kf, Kd) < 1e-13
    Phi = np.conj(Kf)
    B = nfft.dense_B(x, p)
    Ks = Kd.conj().T
    assert rel(Phi @ B.T, (B @ Ks).T) < 1e-13
    assert rel(B.T @ Phi, (Ks @ B).T) < 1e-13


def _tiny_problem(seed=31, d=1):
    g = W.rng(seed)
    if d == 1:
        p = nfft.Params((8,), 2.0, 2)
        x = W.uniform_nodes(g, 22, 1)
    else:
        p = nfft.Params((4, 4), 2.0, 1)
        x = W.uniform_nodes(g, 30, 2)
    return x, p


@pytest.mark.parametrize("d", [1, 2])
def test_separability_dense_problem_equals_per_column_solutions(d):
    """(3.29)-(3.30): min ||K^*B - I||_F^2 + lambda ||B||_F^2 over all entries of B on the
    sparsity pattern at once equals the per-l solutions."""
    x, p = _tiny_problem(d=d)
    rho = 1e-6
    mem = bopt.Members(x, p)
    Ks = _dense_K(x, p).conj().T                     # K^* = F D A^*, (G x N)
    G = Ks.shape[0]
    pairs = [(j, l) for l in range(G) for j in mem.of(l)[0]]
    # vec(K^* B): entry (s, l) = sum_j Ks[s, j] B[j, l]
    nvar = len(pairs)
    Amat = np.zeros((G * G, nvar), dtype=np.complex128)
    for c, (j, l) in enumerate(pairs):
        Amat[np.arange(G) * G + l, c] = Ks[:, j]
    col_norm2 = np.real(np.sum(np.abs(Ks) ** 2, axis=0))   # ||L_l e_j||^2 = column norm of K^*
    lam = rho * np.mean(col_norm2)
    big = np.vstack([Amat, np.sqrt(lam) * np.eye(nvar)])
    rhs = np.concatenate([np.eye(G).ravel(), np.zeros(nvar)])
    sol = np.linalg.lstsq(big, rhs, rcond=None)[0]
    rows, _ = bopt.bopt_rows(x, p, rho, route="E", members=mem)
    Bd = bopt.dense_from_rows(x, rows, p)
    ref = np.array([Bd[j, l] for (j, l) in pairs])
    assert rel(ref, sol) < 1e-9


@pytest.mark.parametrize("route", ["E", "R", "G"])
def test_optimality_conditions(route):
    """Normal equations of the ridge problem: L^*(L b - e_l) + lambda b = 0 (P8)."""
    x, p = _tiny_problem(seed=32)
    rho = 1e-6
    mem = bopt.Members(x, p)
    for l in range(mem.G):
        js, _, _ = mem.of(l)
        if len(js) == 0:
            continue
        b = bopt.ROUTES[route](x, l, js, p, rho)
        L = bopt.L_matrix(x, js, p)
        e = np.zeros(L.shape[0]); e[l] = 1
        lam = rho * np.real(np.trace(L.conj().T @ L)) / len(js)
        resid = L.conj().T @ (L @ b - e) + lam * b
        assert np.linalg.norm(resid) <= 1e-7 * np.linalg.norm(L.conj().T @ e)


@pytest.mark.parametrize("nodes,rho", [("jittered", 1e-6), ("jittered", 1e-10), ("uniform", 1e-6)])
def test_three_routes_agree(nodes, rho):
    """Routes E, R and G solve the same ridge problem.  The local problems carry more nodes than
    their band resolves, so cond(L_l^* L_l + lambda I) ~ 1/rho and the large least-squares
    residual makes every route accurate to ~ eps/rho only; a wrong term in any route would show
    as an O(1) difference."""
    g = W.rng(33)
    p = nfft.Params((16,), 2.0, 3)
    x = W.jittered_nodes(g, 48) if nodes == "jittered" else W.uniform_nodes(g, 48, 1)
    mem = bopt.Members(x, p)
    rE, _ = bopt.bopt_rows(x, p, rho, "E", members=mem)
    rR, _ = bopt.bopt_rows(x, p, rho, "R", members=mem)
    rG, _ = bopt.bopt_rows(x, p, rho, "G", members=mem)
    tol = 100 * 2.2e-16 / rho
    assert rel(rR, rE) < tol and rel(rG, rE) < tol


def test_three_routes_agree_2d():
    g = W.rng(34)
    p = nfft.Params((6, 8), 2.0, 2)
    x = W.uniform_nodes(g, 60, 2)
    mem = bopt.Members(x, p)
    rE, _ = bopt.bopt_rows(x, p, 1e-6, "E", members=mem)
    rG, _ = bopt.bopt_rows(x, p, 1e-6, "G", members=mem)
    rR, _ = bopt.bopt_rows(x, p, 1e-6, "R", members=mem)
    assert rel(rG, rE) < 1e-8 and rel(rR, rE) < 1e-8


def test_single_member_closed_form():
    """|I(l)| = 1: b = <L e, e_l> / (||L e||^2 + lambda), a scalar projection."""
    p = nfft.Params((8,), 2.0, 2)
    x = np.array([[0.013], [0.26], [-0.31]])     # well separated: some grid indices see one node
    mem = bopt.Members(x, p)
    found = 0
    for l in range(mem.G):
        js, _, _ = mem.of(l)
        if len(js) != 1:
            continue
        found += 1
        c = bopt.L_matrix(x, js, p)[:, 0]
        lam = 1e-4 * np.real(np.vdot(c, c))
        expect = np.conj(c[l]) / (np.real(np.vdot(c, c)) + lam)
        for route in "ERG":
            assert abs(bopt.ROUTES[route](x, l, js, p, 1e-4)[0] - expect) < 1e-12 * abs(expect)
    assert found > 0


def test_frobenius_monotone_and_rank_bound():
    """(3.34): the optimised B never does worse than B on the ridge objective, and the
    objective is bounded below by M_sigma - M since rank(K^*B) <= M."""
    for d in (1, 2):
        x, p = _tiny_problem(seed=35, d=d)
        B = nfft.dense_B(x, p)
        rho = 1e-9
        rows, _ = bopt.bopt_rows(x, p, rho, "E")
        Bo = bopt.dense_from_rows(x, rows, p)
        f_B = bopt.frobenius_objective(x, B, p)
        f_O = bopt.frobenius_objective(x, Bo, p)
        Ks = _dense_K(x, p).conj().T
        lam = rho * np.mean(np.real(np.sum(np.abs(Ks) ** 2, axis=0)))
        assert f_O ** 2 + lam * np.sum(np.abs(Bo) ** 2) <= f_B ** 2 + lam * np.sum(np.abs(B) ** 2) + 1e-9
        Gs, P = int(np.prod(p.Ms)), int(np.prod(p.M))
        assert f_O ** 2 >= Gs - P - 1e-9
        assert f_B ** 2 >= Gs - P - 1e-9


def test_apply_equals_dense_product_and_is_adjoint_of_inverse_adjoint():
    for d in (1, 2):
        x, p = _tiny_problem(seed=36, d=d)
        rows, _ = bopt.bopt_rows(x, p, 1e-8, "G")
        Bo = bopt.dense_from_rows(x, rows, p)
        g = W.rng(37)
        f = W.complex_normal(g, (x.shape[0],))
        D, F = nfft.dense_D(p), nfft.dense_F(p)
        h = bopt.apply(x, f, rows, p)
        assert rel(h.ravel(), D.conj().T @ F.conj().T @ Bo.conj().T @ f) < 1e-13
        hh = W.complex_normal(g, p.M)
        ff = bopt.apply_adjoint(x, hh, rows, p)
        assert rel(ff, Bo @ F @ D @ hh.ravel()) < 1e-13
        assert abs(np.vdot(f, ff) - np.vdot(h, hh)) < 1e-12 * abs(np.vdot(f, ff))


def test_optimisation_improves_reconstruction_jittered():
    """Example 3.23 qualitatively: for jittered nodes with N = 2M the modified adjoint
    reconstructs fhat far better than the scaled plain adjoint (no figure data: the size of the
    error is reported, not pinned)."""
    g = W.rng(38)
    M, N = 64, 128
    p = nfft.Params((M,), 2.0, 4)
    x = W.jittered_nodes(g, N)
    fh = W.complex_normal(g, (M,))
    f = direct.ndft(x, fh)
    rows, _ = bopt.bopt_rows(x, p, 1e-12, "R")
    e_opt = rel(bopt.apply(x, f, rows, p), fh)
    e_plain = rel(nfft.adjoint(x, f, p) / N, fh)
    assert e_opt < 1e-3 and e_opt < 1e-2 * e_plain


# ------------------------------------------------------------------ gradients

@pytest.mark.parametrize("d", [1, 2])
def test_node_gradient_matches_finite_differences(d):
    g = W.rng(41 + d)
    M = (16,) if d == 1 else (8, 10)
    p = nfft.Params(M, 2.0, 4)
    x = W.uniform_nodes(g, 7, d)
    fh = W.complex_normal(g, (2,) + M)
    gf = W.complex_normal(g, (2, 7))
    an = grad.nfft_grad_x(x, fh, gf, p)

    def loss(xx):
        return np.sum(np.real(np.conj(gf) * nfft.trafo(xx, fh, p)))

    h = 1e-7
    fd = np.zeros_like(an)
    for j in range(x.shape[0]):
        for t in range(d):
            xp = x.copy(); xp[j, t] += h
            xm = x.copy(); xm[j, t] -= h
            fd[j, t] = (loss(xp) - loss(xm)) / (2 * h)
    assert np.max(np.abs(fd - an)) < 1e-6 * np.max(np.abs(an))
    # and the NFFT derivative approximates the exact derivative of the trigonometric sum
    exact = np.sum(np.real(np.conj(gf)[:, :, None] * direct.ndft_grad_x(x, fh)), axis=0)
    assert np.max(np.abs(exact - an)) < 1e-4 * np.max(np.abs(exact))


# ------------------------------------------------------------------ Dirichlet kernel (Remark 3.19)

def test_dirichlet_kernel_closed_form():
    """With w_hat = 1 for |k| < M/2 and the k = -M/2 entry zeroed, K(y) = D_{M/2-1}(y) / M_sigma,
    D_{M/2-1}(y) = sin((M-1) pi y) / sin(pi y) (3.23); its value at 0 is (M-1)/M_sigma."""
    M, Ms = 20, 40
    p = nfft.Params((M,), 2.0, 3, kernel="dirichlet")
    y = np.linspace(-0.49, 0.49, 97) + 1e-3
    K = bopt.kernel_K(y[:, None], p)
    closed = np.sin((M - 1) * np.pi * y) / np.sin(np.pi * y) / Ms
    assert np.max(np.abs(K - closed)) <= 1e-14 * np.max(np.abs(closed))
    assert abs(bopt.kernel_K(np.zeros((1, 1)), p)[0] - (M - 1) / Ms) < 1e-15


@pytest.mark.parametrize("d", [1, 2])
def test_dirichlet_routes_agree_and_b_opt_is_real(d):
    """The three routes solve the same Dirichlet problem; the kernel is real and even, so the
    Gram matrix and right-hand side are real and so is B_opt (the real B of (3.27))."""
    g = W.rng(50 + d)
    if d == 1:
        p = nfft.Params((16,), 2.0, 3, kernel="dirichlet")
        x = W.jittered_nodes(g, 48)
    else:
        p = nfft.Params((6, 8), 2.0, 2, kernel="dirichlet")
        x = W.uniform_nodes(g, 60, 2)
    mem = bopt.Members(x, p)
    rE, _ = bopt.bopt_rows(x, p, 1e-6, "E", members=mem)
    rR, _ = bopt.bopt_rows(x, p, 1e-6, "R", members=mem)
    rG, _ = bopt.bopt_rows(x, p, 1e-6, "G", members=mem)
    tol = 100 * 2.2e-16 / 1e-6
    assert rel(rR, rE) < tol and rel(rG, rE) < tol
    assert np.max(np.abs(rE.imag)) <= tol * np.max(np.abs(rE))


def test_dirichlet_apply_zeroes_the_unpaired_frequency_and_reconstructs():
    """The zeroed entry of D^* makes the estimate at k = -M/2 vanish; for jittered nodes with
    N = 4M (Example 3.23's setting) the other coefficients are reconstructed closely (the paper's
    figure carries no numbers: the bound is a loose check, the size is reported in the design)."""
    g = W.rng(60)
    M = 32
    p = nfft.Params((M,), 2.0, 4, kernel="dirichlet")
    x = W.jittered_nodes(g, 4 * M)
    fh = W.complex_normal(g, (M,))
    f = direct.ndft(x, fh)
    rows, _ = bopt.bopt_rows(x, p, 1e-12, "G")
    fc = bopt.apply(x, f, rows, p)
    assert fc[0] == 0
    assert rel(fc[1:], fh[1:]) < 1e-5


# ------------------------------------------------------------------ gradient through B_opt(x)

@pytest.mark.parametrize("d,kernel", [(1, "window"), (1, "dirichlet"), (2, "window")])
def test_bopt_gradient_matches_finite_differences(d, kernel):
    """dL/dx through B_opt(x) by implicit differentiation of the ridge normal equations, against
    central differences of L(x) = Re <c, D^* F^* B_opt(x)^* f> with B_opt recomputed at the moved
    nodes (the membership I(l) does not change for steps this small)."""
    g = W.rng(80 + d)
    M, N = ((12,), 30) if d == 1 else ((6, 8), 40)
    p = nfft.Params(M, 2.0, 3 if d == 1 else 2, kernel=kernel)
    x = W.uniform_nodes(g, N, d)
    f = W.complex_normal(g, (2, N))
    c = W.complex_normal(g, (2,) + M)
    rho = 1e-4

    def L(xx):
        rows, _ = bopt.bopt_rows(xx, p, rho, "G")
        return float(np.real(np.vdot(c, bopt.apply(xx, f, rows, p))))

    an = grad.bopt_grad_x(x, f, c, p, rho)
    fd = np.zeros_like(an)
    h = 1e-6
    for j in range(N):
        for t in range(d):
            xp = x.copy()
            xp[j, t] += h
            xm = x.copy()
            xm[j, t] -= h
            fd[j, t] = (L(xp) - L(xm)) / (2 * h)
    assert rel(an, fd) < 1e-6


# ------------------------------------------------------------------ ansatz 1 (Section 3.2.1, Algorithm 3.10)

from oracle import ansatz1 as a1  # noqa: E402


def _a1_problem(seed, N, M, sigma=2.0, m=3, kernel="window"):
    g = W.rng(seed)
    return W.jittered_nodes(g, N), nfft.Params((M,), sigma, m, kernel=kernel)


@pytest.mark.parametrize("kernel,sigma", [("window", 2.0), ("dirichlet", 2.0), ("window", 1.25)])
def test_ansatz1_K_is_the_dense_factor_product(kernel, sigma):
    """(3.14): K = A D^* F^* entry by entry, with F in FFT row order and the inverse's D; the
    column route through e^{2 pi i k x_h} agrees."""
    x, p = _a1_problem(70, 21, 16, sigma, 2, kernel)
    K = a1.K_matrix(x, p)
    Kd = direct.ndft_matrix(x, p.M) @ np.diag(p.deconv_inv_full().ravel()) @ nfft.dense_F(p).conj().T
    assert rel(K, Kd) < 1e-13
    cols = np.array([0, 3, p.Ms[0] - 1, p.Ms[0] // 2])
    assert rel(a1.K_columns(x, cols, p), K[:, cols]) < 1e-13


def test_ansatz1_dirichlet_K_closed_form():
    """Remark 3.11 / (3.23): with the Dirichlet kernel K_j's entries are
    D_{M/2-1}(x_h - l/M_sigma) / M_sigma, D_{M/2-1}(y) = sin((M-1) pi y) / sin(pi y)."""
    x, p = _a1_problem(71, 13, 20, 2.0, 2, "dirichlet")
    K = a1.K_matrix(x, p)
    Ms = p.Ms[0]
    lpos = np.arange(Ms)
    y = x[:, 0][:, None] - np.where(lpos < Ms // 2, lpos, lpos - Ms)[None, :] / Ms
    closed = np.sin((p.M[0] - 1) * np.pi * y) / np.sin(np.pi * y) / Ms
    assert np.max(np.abs(K - closed)) < 1e-13 * np.max(np.abs(closed))


def test_ansatz1_toeplitz_symbol_and_gram_band():
    """A^* A is Toeplitz with symbol P(q) = sum_h e^{2 pi i q x_h}; the band of K^* K built from
    P and R_d by direct sums equals the band read off the dense K^* K, for sigma = 2 and sigma < 2
    (where 2M - 1 frequencies exceed M_sigma)."""
    for kernel, sigma in (("window", 2.0), ("dirichlet", 2.0), ("window", 1.5)):
        x, p = _a1_problem(72, 19, 16, sigma, 3, kernel)
        A = direct.ndft_matrix(x, p.M)
        AhA = A.conj().T @ A
        P = a1.toeplitz_symbol(x, p)
        M = p.M[0]
        k = np.arange(M)
        expect = P[(k[None, :] - k[:, None]) + M - 1]
        assert rel(AhA, expect) < 1e-13
        S = a1.gram_band(x, p)
        Sd = a1.gram_band_direct(a1.K_matrix(x, p), p)
        assert rel(S, Sd) < 1e-12


@pytest.mark.parametrize("kernel,rho", [("window", 0.0), ("window", 1e-8), ("dirichlet", 0.0), ("dirichlet", 1e-6)])
def test_ansatz1_routes_agree_and_stationarity(kernel, rho):
    """Routes E (lstsq on the definition) and T (Toeplitz Gram, normal equations) agree, and
    each y_j satisfies K_j^* (K_j y_j - e_j) + lambda_j y_j = 0 on I(x_j)."""
    x, p = _a1_problem(73, 24, 64, 2.0, 3, kernel)
    K = a1.K_matrix(x, p)
    rE = a1.rows_E(x, p, rho, K=K)
    rT = a1.rows_T(x, p, rho)
    assert rel(rT, rE) < 1e-8
    idx, mem = a1.stencil(x, p)
    for j in range(x.shape[0]):
        t = np.nonzero(mem[j])[0]
        Kj = K[:, idx[j, t]]
        y = np.conj(rE[j, t])
        lam = rho * np.sum(np.abs(Kj) ** 2) / len(t)
        e = np.zeros(x.shape[0])
        e[j] = 1.0
        grad_ = Kj.conj().T @ (Kj @ y - e) + lam * y
        assert np.linalg.norm(grad_) < 1e-9 * np.linalg.norm(Kj.conj().T @ e)
        assert np.all(rE[j, ~mem[j]] == 0)


def test_ansatz1_columns_split_the_frobenius_problem():
    """(3.18)-(3.19): minimising ||K B^* - M I||_F jointly over every nonzero of B^* (one stacked
    least-squares problem) gives the per-node solutions."""
    x, p = _a1_problem(74, 9, 32, 2.0, 2)
    K = a1.K_matrix(x, p)
    idx, mem = a1.stencil(x, p)
    N, Mv = x.shape[0], p.M[0]
    cols = [(j, t) for j in range(N) for t in np.nonzero(mem[j])[0]]
    # vec(K B^*): entry (h, j) = sum_t K[h, idx[j,t]] B^*[idx[j,t], j]
    Big = np.zeros((N * N, len(cols)), dtype=np.complex128)
    for c, (j, t) in enumerate(cols):
        Big[np.arange(N) * N + j, c] = K[:, idx[j, t]]
    target = (Mv * np.eye(N)).ravel().astype(np.complex128)
    sol = np.linalg.lstsq(Big, target, rcond=None)[0]
    rows = a1.rows_E(x, p, 0.0, K=K)
    per = np.array([Mv * np.conj(rows[j, t]) for (j, t) in cols])
    assert rel(sol, per) < 1e-9


def test_ansatz1_objective_monotone_rank_bound_and_underdetermined_gain():
    """Example 3.13's findings as inequalities: the optimised B^* never does worse than the window's
    on (3.24) nor than random perturbations of itself; for M < N no B reaches below the rank bound
    M sqrt(N - M) (K B^* has rank <= M), and the optimum sits at it; for M = 4N the optimisation cuts
    the norm by orders of magnitude."""
    g = W.rng(75)
    N = 32
    x = W.jittered_nodes(g, N)
    for M, m in ((8, 2), (16, 2), (128, 4)):
        p = nfft.Params((M,), 2.0, m)
        K = a1.K_matrix(x, p)
        rows = a1.rows_E(x, p, 0.0, K=K)
        o = a1.objective(x, rows, p, K=K)
        o_plain = a1.objective(x, a1.plain_rows(x, p), p, K=K)
        assert o <= o_plain
        _, mem = a1.stencil(x, p)
        for _ in range(3):
            pert = rows + 1e-3 * np.abs(rows).max() * W.complex_normal(g, rows.shape) * mem
            assert o <= a1.objective(x, pert, p, K=K)
        if M < N:
            bound = M * np.sqrt(N - M)
            assert o >= bound * (1 - 1e-12)
            assert o <= bound * 1.05
        else:
            assert o < 1e-2 * o_plain


def test_ansatz1_reconstruction_and_inverse_adjoint_example_3_14():
    """Example 3.14 / 3.16 setting (Dirichlet kernel, sigma = 2, jittered nodes, M = 4N, m = 4):
    A f_check reproduces f = A fhat closely, and f_tilde = (1/M) B_opt F D (A^* f) of Remark 3.15
    reproduces f; both estimates are adjoint to each other; B_opt is real."""
    g = W.rng(76)
    N = 32
    M = 4 * N
    x = W.jittered_nodes(g, N)
    p = nfft.Params((M,), 2.0, 4, kernel="dirichlet")
    rows = a1.rows_E(x, p, 0.0)
    assert np.max(np.abs(rows.imag)) < 1e-9 * np.max(np.abs(rows))
    fh = W.complex_normal(g, (M,))
    f = direct.ndft(x, fh)
    fc = bopt.apply(x, f, rows, p)
    r_inv = rel(direct.ndft(x, fc), f)
    ft = bopt.apply_adjoint(x, direct.ndft_adjoint(x, f, p.M), rows, p)
    r_adj = rel(ft, f)
    r_plain = rel(direct.ndft(x, nfft.adjoint(x, f, nfft.Params((M,), 2.0, 4)) / M), f)
    assert r_inv < 1e-2 and r_adj < 1e-2 and r_inv < 1e-1 * r_plain
    hh = W.complex_normal(g, (M,))
    assert abs(np.vdot(f, bopt.apply_adjoint(x, hh, rows, p)) - np.vdot(fc, hh)) < 1e-12 * np.linalg.norm(f) * np.linalg.norm(hh) * np.abs(rows).max() * M


# ------------------------------------------------------------------ Theorem 4.3 (frame link, §4.2.1)

def _frame_terms(M, sigma, m, N, seed):
    """The quantities of Theorem 4.3 from the oracle's matrices: B (2.6); Phi = Phi_l2 of Section 4.2,
    conj K(x_j - l / M_sigma) with the kernel K of (3.15); Psi = (psi_l(k)) of the discrete frames,
    e^{-2 pi i k l / M_sigma} / (M_sigma w_hat(-k)); c = B^* f (the adjoint NFFT's coefficients) and
    d = Phi^+ f (the frame approximation's); and the vector of 1 / w_hat(-k)."""
    p = nfft.Params((M,), sigma, m)
    g = W.rng(seed)
    x = g.uniform(-0.5, 0.5, N)
    Ms = p.Ms[0]
    B = nfft.dense_B(x, p)                                    # columns in FFT order of l
    lpos = np.arange(Ms)
    lval = np.where(lpos < Ms // 2, lpos, lpos - Ms)
    Phi = np.conj(bopt.kernel_K_1d((x[:, None] - lval[None, :] / Ms).ravel(), p, 0)).reshape(N, Ms)
    D = p.deconv(0)                                           # D_k = 1 / (M_sigma w_hat(-k))
    k = direct.centred(M)
    Psi = D[:, None] * np.exp(-2j * np.pi * np.outer(k, lval) / Ms)
    w_inv = Ms * D
    f = W.complex_normal(g, (N,))
    Pinv = np.linalg.pinv(Phi)
    return dict(B=B, Phi=Phi, Psi=Psi, w_inv=w_inv, f=f, Pinv=Pinv, c=B.T @ f, d=Pinv @ f, Ms=Ms, N=N)


@pytest.mark.parametrize("M,sigma,N,case", [(16, 2.0, 10, "ii"), (16, 2.0, 12, "ii"),
                                            (16, 1.0, 40, "i"), (24, 1.0, 60, "i")])
def test_theorem_4_3_frame_distance_bounds(M, sigma, N, case):
    """Theorem 4.3: ||h~ - h~~||_2 with h~ = Psi B^* f and h~~ = Psi Phi^+ f is at most
    ||w_hat||_2 / sqrt(M_sigma) times ||Phi B^* - I_N||_F ||Phi^+ f||_2 (4.11, M_sigma < N) or
    ||B^* Phi - I_{M_sigma}||_F ||Phi^+ f||_2 (4.12, M_sigma > N).  Pinned with the proof's exact
    steps: ||Psi||_F equals ||w_hat||_2 / sqrt(M_sigma), and c - d equals
    Phi^+ (Phi B^* - I) f (full column rank of Phi: sigma = 1, N > M_sigma) or
    (B^* Phi - I) Phi^+ f (full row rank: N < M; with sigma = 2 Phi has rank at most M < M_sigma,
    so case (i) needs sigma = 1)."""
    t = _frame_terms(M, sigma, 3, N, seed=90 + N)
    Psi, c, d, Ms = t["Psi"], t["c"], t["d"], t["Ms"]
    fac = np.linalg.norm(t["w_inv"]) / np.sqrt(Ms)
    assert np.linalg.norm(Psi) == pytest.approx(fac, rel=1e-12)
    lhs = np.linalg.norm(Psi @ (c - d))
    if case == "i":
        assert Ms < N and np.linalg.matrix_rank(t["Phi"]) == Ms
        E = t["Phi"] @ t["B"].T - np.eye(N)
        assert rel(c - d, t["Pinv"] @ (E @ t["f"])) < 1e-10
    else:
        assert Ms > N and np.linalg.matrix_rank(t["Phi"]) == N
        E = t["B"].T @ t["Phi"] - np.eye(Ms)
        assert rel(c - d, E @ d) < 1e-10
    bound = fac * np.linalg.norm(E) * np.linalg.norm(d)
    assert lhs <= bound * (1 + 1e-12)
