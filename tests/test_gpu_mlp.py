"""GPU parity of the parameter predictor: network forward, loss gradient and
Adam step against the FP64 numpy oracle, and the moment features against the
oracle's moments of the same random-phase vectors."""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.mlp as OM
from topi import random_phase_block, topi_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1803_02156_amd as P
    P.load()
    return P


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (B, OM.D_IN))
    T = rng.standard_normal((B, OM.D_OUT))
    theta = OM.init_params(seed)
    theta[OM.SHAPES[0][0] * OM.SHAPES[0][1]:][:128] = rng.uniform(-0.1, 0.1, 128)   # nonzero b1
    return X.astype(np.float32), T.astype(np.float32), theta.astype(np.float32)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("B", [1, 7, 64, 200, 2000])
def test_forward_matches_oracle(P, B):
    X, _, theta = _batch(B, B)
    y = P.chebfd_mlp_forward(_cuda(theta), _cuda(X)).cpu().numpy()
    ref, _ = OM.forward(theta.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(y - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("B", [1, 33, 500, 2000])
def test_grad_matches_oracle(P, B):
    X, T, theta = _batch(B, 100 + B)
    loss, g = P.chebfd_mlp_grad(_cuda(theta), _cuda(X), _cuda(T))
    rl, rg = OM.gradient(theta.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert abs(loss.item() - rl) <= 1e-4 * abs(rl)
    g = g.cpu().numpy()
    # per parameter block, relative to the block's largest gradient
    at = 0
    for s in OM.SHAPES:
        k = int(np.prod(s))
        scale = max(np.max(np.abs(rg[at:at + k])), 1e-30)
        assert np.max(np.abs(g[at:at + k] - rg[at:at + k])) <= 1e-4 * scale, s
        at += k


def test_grad_is_reproducible(P):
    X, T, theta = _batch(300, 5)
    a = P.chebfd_mlp_grad(_cuda(theta), _cuda(X), _cuda(T))[1]
    b = P.chebfd_mlp_grad(_cuda(theta), _cuda(X), _cuda(T))[1]
    assert torch.equal(a, b)


def test_adam_matches_oracle_over_steps(P):
    X, T, theta = _batch(128, 9)
    p = _cuda(theta)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    rt, rm, rv = theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size)
    for step in range(1, 4):
        g = torch.from_numpy(np.random.default_rng(step).standard_normal(theta.size).astype(np.float32)).cuda()
        P.chebfd_mlp_adam(p, g, m, v, step, lr=1e-2)
        # the kernel receives the hyper-parameters as float32: give the oracle the same values
        f32 = lambda x: float(np.float32(x))  # noqa: E731
        rt, rm, rv = OM.adam(rt, g.cpu().numpy().astype(np.float64), rm, rv, step, lr=f32(1e-2),
                             beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-8))
        assert np.max(np.abs(p.cpu().numpy() - rt)) <= 1e-6 + 1e-5 * np.max(np.abs(rt))
        assert np.max(np.abs(v.cpu().numpy() - rv)) <= 1e-5 * np.max(rv)


def test_training_reduces_loss(P):
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (512, OM.D_IN)).astype(np.float32)
    T = np.stack([np.sin(3 * X[:, 0]) + X[:, 1], X[:, 2] * X[:, 3]], axis=1).astype(np.float32)
    p = _cuda(OM.init_params(1).astype(np.float32))
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    x, t = _cuda(X), _cuda(T)
    first = None
    for step in range(1, 201):
        loss, g = P.chebfd_mlp_grad(p, x, t)
        first = loss.item() if first is None else first
        P.chebfd_mlp_adam(p, g, m, v, step, lr=1e-3)
    assert P.chebfd_mlp_grad(p, x, t)[0].item() < 0.2 * first


@pytest.mark.parametrize("prec", [0, 1])
def test_features_match_oracle(P, prec):
    H = topi_csr(8, 6, 5, m=1.0, W=1.0, seed=77)
    n = len(H[0]) - 1
    M = P.chebfd_matrix_build(*H, prec=prec)
    f, cnt, al, be = P.chebfd_features(M, -0.3, 0.3, seed=11)
    lo, hi = O.gershgorin_bounds(H)
    ral, rbe = O.scale_factors(lo, hi)
    # bounds from the stored matrix values (c64 in mixed precision)
    rel = 1e-15 if prec == 0 else 1e-6
    assert abs(al - ral) < rel * ral and abs(be - rbe) < rel
    X = random_phase_block(n, 16, 11)
    _, eta, nu = O.chebyshev_filter(H, ral, rbe, np.zeros(129), X, 16)
    mu = np.real(np.sum(O.kpm_moments(eta, nu), axis=1)) / (n * 16)
    tol = 1e-6 if prec == 0 else 2e-4          # features are stored in FP32
    assert np.max(np.abs(f[1:256] - mu[1:])) < tol
    assert abs(mu[0] - 1.0) < 1e-12 and f[0] == np.float32(np.log10(n) / 8.0)   # slot 0: the size
    assert abs(f[256] - (ral * -0.3 + rbe)) < 1e-7 and abs(f[257] - (ral * 0.3 + rbe)) < 1e-7
    ref_cnt = O.count_estimate(O.kpm_moments(eta, nu), n, ral * -0.3 + rbe, ral * 0.3 + rbe)
    assert abs(cnt - ref_cnt) < (1e-9 if prec == 0 else 1e-2) * max(1.0, abs(ref_cnt))
