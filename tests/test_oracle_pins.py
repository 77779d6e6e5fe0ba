"""Pins for the FP64 CPU oracle: each part is checked against something other than
itself -- closed forms, an independent definition, dense LAPACK diagonalisation
or brute force on tiny inputs."""
import numpy as np
import pytest

import oracle as O
from topi import csr_to_dense, diag_csr, random_phase_block, topi_csr
from tests.bloch import bloch_spectrum


# --------------------------------------------------------------------------- coefficients
def _cheb_quadrature(f, n_p, N=400000):
    """(2 - delta_p0)/pi int_0^pi f(cos t) cos(pt) dt by the midpoint rule in t."""
    t = np.pi * (np.arange(N) + 0.5) / N
    ft = f(np.cos(t))
    p = np.arange(n_p + 1)
    c = np.array([np.mean(ft * np.cos(k * t)) for k in p]) * 2.0
    c[0] /= 2.0
    return c


@pytest.mark.parametrize("a,b", [(-0.3, 0.2), (-0.05, 0.05), (0.1, 0.9), (-0.99, -0.5)])
def test_window_coefficients_match_quadrature(a, b):
    c = O.window_coefficients(a, b, 60)
    q = _cheb_quadrature(lambda x: ((x >= a) & (x <= b)).astype(float), 60)
    assert np.max(np.abs(c - q)) < 2e-5


def test_window_symmetric_interval_odd_terms_vanish():
    c = O.window_coefficients(-0.2, 0.2, 101)
    assert np.max(np.abs(c[1::2])) < 1e-15
    assert abs(c[0] - (np.arccos(-0.2) - np.arccos(0.2)) / np.pi) < 1e-15


def test_jackson_equals_autocorrelation_of_sine_sequence():
    # independent definition: g_p = sum_v a_v a_{v+p} for the unit-norm a_v ~ sin(pi (v+1)/(M+1))
    for n_p in (5, 40, 199):
        M = n_p + 1
        a = np.sin(np.pi * (np.arange(M) + 1) / (M + 1))
        a /= np.linalg.norm(a)
        ac = np.array([np.dot(a[:M - p], a[p:]) for p in range(M)])
        assert np.max(np.abs(O.jackson_damping(n_p) - ac)) < 1e-14


def test_jackson_properties():
    g = O.jackson_damping(200)
    assert g[0] == pytest.approx(1.0, abs=1e-15)
    assert np.all(g > 0) and np.all(np.diff(g) < 0)


@pytest.mark.parametrize("a,b,n_p", [(-0.1, 0.1, 200), (-0.4, 0.3, 57), (0.5, 0.95, 400)])
def test_damped_window_polynomial_between_0_and_1(a, b, n_p):
    # Jackson damping keeps the polynomial approximation of an indicator in [0, 1]
    gam = O.jackson_damping(n_p) * O.window_coefficients(a, b, n_p)
    x = np.linspace(-1, 1, 100001)
    pv = np.cos(np.outer(np.arccos(x), np.arange(n_p + 1))) @ gam
    assert pv.min() > -1e-12 and pv.max() < 1 + 1e-12


def test_damped_window_converges_to_indicator():
    a, b = -0.2, 0.3
    inside, outside = 0.05, 0.6
    prev_in, prev_out = 0.0, 1.0
    for n_p in (50, 200, 800):
        gam = O.jackson_damping(n_p) * O.window_coefficients(a, b, n_p)
        pv = np.cos(np.outer(np.arccos([inside, outside]), np.arange(n_p + 1))) @ gam
        assert pv[0] > prev_in - 1e-12 and pv[1] < prev_out + 1e-12
        prev_in, prev_out = pv
    assert prev_in > 0.999 and prev_out < 1e-6


# --------------------------------------------------------------------------- scaling
def test_gershgorin_brute_force_and_contains_spectrum():
    H = topi_csr(3, 4, 3, m=1.2, W=2.5, seed=8, dilution=0.2, dilution_seed=1)
    A = csr_to_dense(*H)
    c = np.real(np.diag(A))
    r = np.sum(np.abs(A), axis=1) - np.abs(np.diag(A))
    lo, hi = O.gershgorin_bounds(H)
    assert lo == pytest.approx(np.min(c - r), abs=1e-13)
    assert hi == pytest.approx(np.max(c + r), abs=1e-13)
    e = np.linalg.eigvalsh(A)
    assert lo <= e[0] and e[-1] <= hi


def test_gershgorin_topi_closed_form():
    from topi import site_disorder
    m, W, t = 1.0, 1.0, 1.0
    H = topi_csr(4, 4, 4, m=m, W=W, t=t, seed=5)
    lo, hi = O.gershgorin_bounds(H)
    V = site_disorder(64, W, 5)
    assert hi == pytest.approx(np.max(np.abs(m + V)) + 6 * t, abs=1e-14)
    assert lo == -hi
    alpha, beta = O.scale_factors(lo, hi)
    assert beta == 0.0 and alpha * hi == pytest.approx(1.0, abs=1e-15)


def test_scale_factors_map_to_unit_interval():
    al, be = O.scale_factors(-3.0, 5.0)
    assert al * -3.0 + be == pytest.approx(-1.0) and al * 5.0 + be == pytest.approx(1.0)
    with pytest.raises(ValueError):
        O.scale_factors(1.0, 1.0)


# --------------------------------------------------------------------------- filter (Alg. 1/2)
@pytest.mark.parametrize("n_s,n_b,n_p", [(4, 2, 50), (6, 6, 3), (3, 1, 2), (2, 2, 1), (2, 1, 0)])
def test_filter_chebyshev_identity(n_s, n_b, n_p):
    # H = diag(cos t_j), alpha = 1, beta = 0:  T_p(H) x = cos(p t) x exactly
    n = 300
    t = np.linspace(0.003, np.pi - 0.003, n)
    H = diag_csr(np.cos(t))
    gam = np.random.default_rng(n_p).standard_normal(n_p + 1)
    X = random_phase_block(n, n_s, 1)
    Y, eta, nu = O.chebyshev_filter(H, 1.0, 0.0, gam, X, n_b)
    P = np.arange(n_p + 1)
    C = np.cos(np.outer(t, P))               # C[i, p] = cos(p t_i) = T_p(cos t_i)
    assert np.max(np.abs(Y - (C @ gam)[:, None] * X)) < 1e-12 * max(1, n_p)
    w = np.abs(X) ** 2
    for p in range(1, n_p + 1):
        assert np.allclose(eta[p], (C[:, p] * C[:, p - 1]) @ w, atol=1e-11)
        assert np.allclose(nu[p], (C[:, p - 1] ** 2) @ w, atol=1e-11)


@pytest.mark.parametrize("dims,W,n_b", [((4, 4, 3), 2.0, 4), ((3, 3, 4), 0.5, 8)])
def test_filter_equals_dense_polynomial(dims, W, n_b):
    # p(H~) X through the eigendecomposition: an independent evaluation of the filter
    H = topi_csr(*dims, m=1.0, W=W, seed=4)
    A = csr_to_dense(*H)
    lo, hi = O.gershgorin_bounds(H)
    al, be = O.scale_factors(lo, hi)
    gam = O.filter_coefficients(-0.4, 0.25, al, be, 90)
    X = random_phase_block(A.shape[0], 8, 5)
    Y, eta, nu = O.chebyshev_filter(H, al, be, gam, X, n_b)
    L, V = np.linalg.eigh(A)
    pl = np.cos(np.outer(np.arccos(np.clip(al * L + be, -1, 1)), np.arange(91))) @ gam
    Yd = V @ (pl[:, None] * (V.conj().T @ X))
    assert np.max(np.abs(Y - Yd)) < 1e-12


def test_moments_equal_dense_spectral_sums():
    H = topi_csr(4, 3, 3, m=1.0, W=1.0, seed=6)
    A = csr_to_dense(*H)
    lo, hi = O.gershgorin_bounds(H)
    al, be = O.scale_factors(lo, hi)
    n_p = 64
    X = random_phase_block(A.shape[0], 4, 7)
    _, eta, nu = O.chebyshev_filter(H, al, be, np.ones(n_p + 1), X, 4)
    mu = O.kpm_moments(eta, nu)
    L, V = np.linalg.eigh(A)
    w = np.abs(V.conj().T @ X) ** 2
    ref = np.cos(np.outer(np.arange(2 * n_p), np.arccos(al * L + be))) @ w
    assert np.max(np.abs(mu - ref)) < 1e-11
    assert np.max(np.abs(mu.imag)) < 1e-11


def test_moments_odd_trace_vanishes_for_chiral_matrix():
    # trace moments (all unit vectors) of the chiral Topi matrix: odd ones are zero
    H = topi_csr(3, 3, 3, m=1.0, W=1.0, seed=2)
    n = 108
    lo, hi = O.gershgorin_bounds(H)
    al, be = O.scale_factors(lo, hi)
    _, eta, nu = O.chebyshev_filter(H, al, be, np.ones(21), np.eye(n), 36)
    mu = O.kpm_moments(eta, nu).sum(axis=1)
    assert abs(mu[0] - n) < 1e-12
    assert np.max(np.abs(mu[1::2])) < 1e-10


def test_count_estimate_close_to_exact_count():
    H = topi_csr(6, 6, 6, m=1.0, W=1.0, seed=21)
    A = csr_to_dense(*H)
    n = A.shape[0]
    lo, hi = O.gershgorin_bounds(H)
    al, be = O.scale_factors(lo, hi)
    lam_L, lam_R = -1.0, 1.0
    e = np.linalg.eigvalsh(A)
    exact = np.count_nonzero((e >= lam_L) & (e <= lam_R))
    n_p, R = 200, 16
    X = random_phase_block(n, R, 99)
    _, eta, nu = O.chebyshev_filter(H, al, be, np.ones(n_p + 1), X, 16)
    est = O.count_estimate(O.kpm_moments(eta, nu), n, al * lam_L + be, al * lam_R + be)
    # stochastic trace error ~ sqrt(count / R); plus the smoothing at the window edges
    assert abs(est - exact) < 4 * np.sqrt(exact / R) + 3


# --------------------------------------------------------------------------- SVQB / RR / residuals
def test_svqb_orthonormal_same_span():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((400, 12)) + 1j * rng.standard_normal((400, 12))
    Y[:, 5] *= 1e-6
    Q, nd = O.svqb(Y)
    assert nd == 0
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(12))) < 1e-9
    Q2, _ = O.svqb(Q)
    assert np.max(np.abs(Q2.conj().T @ Q2 - np.eye(12))) < 1e-14
    P1 = Q2 @ Q2.conj().T
    Qy, _ = np.linalg.qr(Y)
    assert np.max(np.abs(P1 - Qy @ Qy.conj().T)) < 1e-10


def test_svqb_drops_dependent_columns():
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((300, 8)) + 1j * rng.standard_normal((300, 8))
    Y[:, 3] = Y[:, 1]
    Y[:, 6] = 2 * Y[:, 0] - Y[:, 2]
    Q, nd = O.svqb(Y)
    assert nd == 2 and Q.shape == (300, 6)
    Q, nd = O.svqb(Q)
    assert nd == 0
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(6))) < 1e-13
    # the kept directions still span the original columns
    assert np.max(np.abs(Y - Q @ (Q.conj().T @ Y))) < 1e-10


def _dft_columns(n, m):
    """m columns of the unitary n-point DFT matrix: orthonormal by construction."""
    j = np.arange(n)[:, None]
    k = np.arange(m)[None, :]
    return np.exp(-2j * np.pi * j * k / n) / np.sqrt(n)


def test_qr_positive_recovers_known_factors():
    # X = V U with V orthonormal and U upper triangular with a positive diagonal:
    # by uniqueness of that factorisation Q = V and R = U
    rng = np.random.default_rng(7)
    n, m = 96, 11
    V = _dft_columns(n, m)[:, rng.permutation(m)]
    U = np.triu(rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m)), 1)
    U += np.diag(rng.uniform(0.5, 3.0, m))
    Q, R = O.qr_positive(V @ U)
    assert np.max(np.abs(Q - V)) < 1e-13
    assert np.max(np.abs(R - U)) < 1e-13


def test_qr_positive_matches_modified_gram_schmidt():
    # an independent algorithm, element by element in plain loops
    rng = np.random.default_rng(8)
    n, m = 14, 5
    X = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    Qg = [[0j] * m for _ in range(n)]
    Rg = [[0j] * m for _ in range(m)]
    W = [[complex(X[i, j]) for j in range(m)] for i in range(n)]
    for k in range(m):
        nrm = sum(abs(W[i][k]) ** 2 for i in range(n)) ** 0.5
        Rg[k][k] = nrm
        for i in range(n):
            Qg[i][k] = W[i][k] / nrm
        for j in range(k + 1, m):
            r = sum(Qg[i][k].conjugate() * W[i][j] for i in range(n))
            Rg[k][j] = r
            for i in range(n):
                W[i][j] -= r * Qg[i][k]
    Q, R = O.qr_positive(X)
    assert np.max(np.abs(Q - np.array(Qg))) < 1e-13
    assert np.max(np.abs(R - np.array(Rg))) < 1e-13
    assert np.all(np.diag(R).imag == 0) and np.all(np.diag(R).real > 0)


def test_qr_orth_drops_dependent_columns():
    rng = np.random.default_rng(9)
    Y = rng.standard_normal((300, 8)) + 1j * rng.standard_normal((300, 8))
    Y[:, 3] = Y[:, 1] * (0.5 - 2j)
    Y[:, 6] = 2 * Y[:, 0] - Y[:, 2]
    Y[:, 5] *= 1e-5          # small but independent: kept
    Q, nd = O.qr_orth(Y)
    assert nd == 2 and Q.shape == (300, 6)
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(6))) < 1e-13
    assert np.max(np.abs(Y - Q @ (Q.conj().T @ Y))) < 1e-10
    # the kept directions are the QR of the independent columns, in order
    Qi, _ = O.qr_positive(Y[:, [0, 1, 2, 4, 5, 7]])
    assert np.max(np.abs(Q - Qi)) < 1e-12


def test_rayleigh_ritz_on_exact_invariant_subspace():
    H = topi_csr(4, 3, 3, m=1.0, W=2.0, seed=12)
    A = csr_to_dense(*H)
    L, V = np.linalg.eigh(A)
    idx = [10, 40, 41, 77]
    rng = np.random.default_rng(0)
    M, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    theta, Z = O.rayleigh_ritz(H, V[:, idx] @ M)
    assert np.max(np.abs(theta - L[idx])) < 1e-12
    r = O.residual_norms(H, Z, theta)
    assert np.max(r) < 1e-12


def test_residual_norms_brute_force():
    H = topi_csr(3, 3, 3, m=1.0, W=1.0, seed=1)
    A = csr_to_dense(*H)
    Z = random_phase_block(108, 3, 3)
    th = np.array([0.1, -0.5, 2.0])
    r = O.residual_norms(H, Z, th)
    Zn = Z / np.linalg.norm(Z, axis=0)
    assert np.allclose(r, np.linalg.norm(A @ Zn - Zn * th, axis=0), rtol=1e-13)


def test_fix_phases():
    Z = random_phase_block(50, 3, 1) * np.array([1.0, 2.0, 3.0])
    Z[7, 1] = 10j
    F = O.fix_phases(Z)
    assert np.allclose(np.abs(F), np.abs(Z))
    assert F[7, 1] == pytest.approx(10.0)


# --------------------------------------------------------------------------- full solve
@pytest.mark.parametrize("dims,W,interval,n_s,n_p,n_b", [
    ((4, 4, 3), 2.0, (-0.8, 0.8), 32, 150, 16),
    ((6, 6, 4), 1.0, (-0.35, 0.35), 32, 200, 32),
])
@pytest.mark.parametrize("orth", ["svqb", "tsqr"])
def test_solve_matches_lapack(dims, W, interval, n_s, n_p, n_b, orth):
    H = topi_csr(*dims, m=1.0, W=W, seed=1001)
    A = csr_to_dense(*H)
    n = A.shape[0]
    e = np.linalg.eigvalsh(A)
    lam_L, lam_R = interval
    ref = e[(e >= lam_L) & (e <= lam_R)]
    res = O.chebfd_solve(H, lam_L, lam_R, n_s, n_p, n_b, random_phase_block(n, n_s, 43),
                         refill_seed=44, orth=orth)
    assert res.status == 0
    assert res.n_found == len(ref) and len(ref) % 2 == 0
    assert np.max(np.abs(np.sort(res.theta[:res.n_found]) - ref)) < 1e-12
    assert np.max(res.resid[:res.n_found]) <= 1e-9
    # residuals recomputed independently from the returned vectors
    Z = res.Z[:, :res.n_found]
    Zn = Z / np.linalg.norm(Z, axis=0)
    assert np.max(np.linalg.norm(A @ Zn - Zn * res.theta[:res.n_found], axis=0)) <= 1e-9


def test_solve_clean_lattice_matches_bloch():
    # clean 16x16x8 lattice (the small configuration's shape), m = t = 1: twelve
    # zero modes, next level |E| ~ 0.39; completeness from the closed form
    dims = (16, 16, 8)
    H = topi_csr(*dims, m=1.0, W=0.0)
    n = 4 * 16 * 16 * 8
    E = bloch_spectrum(*dims, 1.0)
    ref = E[(E >= -0.05) & (E <= 0.05)]
    assert len(ref) == 12
    res = O.chebfd_solve(H, -0.05, 0.05, 32, 200, 32, random_phase_block(n, 32, 43),
                         refill_seed=44)
    assert res.status == 0 and res.n_found == 12
    assert np.max(np.abs(res.theta[:12] - ref)) < 1e-12
    assert np.max(res.resid[:12]) <= 1e-9


def test_solve_small_configuration_matches_shift_invert():
    # Topi-16-16-8, m = W = 1, interval [-0.05, 0.05] in H's units, n_s = n_b = 32,
    # n_p = 200: the eigenvalues nearest 0 from sparse shift-invert Lanczos (ARPACK
    # with a sparse LU), an independent method
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    dims = (16, 16, 8)
    n = 4 * 16 * 16 * 8
    H = topi_csr(*dims, m=1.0, W=1.0, seed=1001)
    A = sp.csr_matrix((H[2], H[1], H[0]), shape=(n, n)).tocsc()
    near0 = np.sort(sla.eigsh(A, k=24, sigma=0.0, which="LM", return_eigenvectors=False))
    ref = near0[np.abs(near0) <= 0.05]
    assert np.abs(near0).max() > 0.05          # the 24 nearest include everything inside
    res = O.chebfd_solve(H, -0.05, 0.05, 32, 200, 32, random_phase_block(n, 32, 43),
                         refill_seed=44)
    assert res.status == 0 and res.n_found == len(ref)
    assert np.max(np.abs(res.theta[:res.n_found] - ref)) < 1e-12
    assert np.max(res.resid[:res.n_found]) <= 1e-9


# Instances whose in-interval Ritz pairs include stable mixtures (residuals just
# under the half width) beside the converged eigenpairs: the solve must stop once
# the converged count repeats and those residuals stall, with the exact count.
STALL_CASES = [
    # dims, m, W, disorder seed, half width, n_p, n_s, most iterations
    ((12, 17, 17), 1.5829323234375885, 0.32055382207121985, 1200002, 0.5856721148945054, 559, 64, 8),
    ((11, 12, 15), 1.8410209481090003, 2.8398561100559334, 1200004, 0.5083305263333662, 342, 96, 12),
]


@pytest.mark.parametrize("dims,m,W,seed,hw,n_p,n_s,max_it", STALL_CASES)
def test_solve_stops_when_unresolved_pairs_stall(dims, m, W, seed, hw, n_p, n_s, max_it):
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    H = topi_csr(*dims, m=m, W=W, seed=seed)
    n = len(H[0]) - 1
    A = sp.csr_matrix((H[2], H[1], H[0]), shape=(n, n)).tocsc()
    near0 = np.sort(sla.eigsh(A, k=40, sigma=0.0, which="LM", return_eigenvectors=False))
    assert np.abs(near0).max() > hw          # the 40 nearest include everything inside
    ref = near0[np.abs(near0) <= hw]
    tr = []
    res = O.chebfd_solve(H, -hw, hw, n_s, n_p, 32, random_phase_block(n, n_s, 43 + seed),
                         refill_seed=43 + seed, max_iter=12, trace=tr)
    assert res.status == 0 and res.iterations <= max_it
    assert res.n_found == len(ref) > 0
    assert np.max(np.abs(np.sort(res.theta[:res.n_found]) - ref)) < 1e-12
    # the pairs that stopped the iteration: in the interval, unconverged, residuals
    # that did not halve over the last iteration
    (_, th1, r1), (_, th2, r2) = tr[-2], tr[-1]
    un1 = r1[(np.abs(th1) <= hw) & (r1 > 1e-9)]
    un2 = r2[(np.abs(th2) <= hw) & (r2 > 1e-9)]
    assert len(un2) == 0 or un2.min() > 0.5 * un1.min()


def test_choose_params_reading():
    # heuristic: n_p = kappa / half width, n_s = 2 n_hat rounded up to a block
    assert O.choose_params(-0.01, 0.01, 47.3, 32, kappa=2.0) == (200, 96)
    assert O.choose_params(-0.5, 0.5, 0.0, 16, kappa=2.0) == (50, 16)           # both floors
    assert O.choose_params(-1e-5, 1e-5, 1e4, 32, kappa=2.0) == (20000, 512)     # both ceilings
    # network outputs are de-standardised logs of n_p delta and n_s / max(2 n_hat, n_b);
    # n_s kept >= 1.2 n_hat
    n_p, n_s = O.choose_params(-0.1, 0.1, 100.0, 32, mlp_out=(0.0, 0.0), t_mean=(np.log(80.0), np.log(0.2)))
    assert n_p == 800 and n_s == 128                                            # 1.2 n_hat = 120 -> 128
    n_p, n_s = O.choose_params(-0.02, 0.06, 100.0, 32, mlp_out=(1.0, -1.0), t_mean=(np.log(10.0), np.log(3.0)),
                               t_std=(np.log(2.0), np.log(2.0)))
    assert n_p == 500 and n_s == 320                                            # 20 / 0.04, 1.5 x 200
    n_p, n_s = O.choose_params(-0.1, 0.1, 3.0, 32, mlp_out=(0.0, 0.0), t_mean=(np.log(20.0), np.log(1.5)))
    assert n_p == 200 and n_s == 64                                             # 2 n_hat < n_b: 1.5 x 32
    # outputs held to the training range [t_lo, t_hi] of the log targets
    kw = dict(t_mean=(np.log(20.0), np.log(1.5)), t_std=(1.0, 1.0), t_lo=(np.log(5.0), 0.0),
              t_hi=(np.log(50.0), np.log(2.0)))
    assert O.choose_params(-0.1, 0.1, 100.0, 32, mlp_out=(5.0, 5.0), **kw) == (500, 416)     # 50 / 0.1, 2 x 200
    assert O.choose_params(-0.1, 0.1, 100.0, 32, mlp_out=(-5.0, -5.0), **kw) == (50, 224)   # 5 / 0.1; 1 x 200
    assert O.choose_params(-0.1, 0.1, 100.0, 32, mlp_out=(0.0, 0.0), **kw) == (200, 320)    # inside: unchanged
