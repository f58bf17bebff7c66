"""Weighted min-sum with damping (the differentiable form of the decoder): pins of
the oracle's forward map and of the plain-PyTorch autograd reference.

Pins: reduction to plain normalized min-sum at beta = 0, alpha = alpha_0; beta = 1
keeps every check message at r^(0) = 0; the iteration-1 closed form; a two-check
path worked by hand through two damped iterations; the PyTorch reference's
forward equal to the oracle's (both precisions) and its autograd gradient equal
to central finite differences of the FP64 oracle away from non-smooth points.
"""

import numpy as np
import pytest
import torch

import oracle
from tests import wbp_reference as ref
from tests.common import bases_for
from workloads import codes
from workloads.configs import WORKLOADS


def _setup(code, wl, shots, p, seed=7, shot0=0):
    ex, ez, sx, sz = oracle.sample(code.hx, code.hz, seed, p, shot0, shots)
    bp, rows = bases_for(code.hz, wl, oracle.build_bases)
    return ex, sx, bp, rows


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_weighted_reduces_to_plain(precision):
    wl = WORKLOADS["bb72_L4_T20"]
    code = codes.bb72()
    ex, sx, bp, rows = _setup(code, wl, 300, 0.06)
    mu = np.full(code.n, oracle.prior_llr(0.06))
    L, T = wl.L, wl.T
    plain = oracle.decode(code.hz, bp, rows, sx, mu, T, alpha=wl.alpha, want_llr=True, precision=precision)
    wa = np.full((T, L), wl.alpha)
    wb = np.zeros((T, L))
    wgt = oracle.decode(code.hz, bp, rows, sx, mu, T, rule=oracle.WNMS, want_llr=True, precision=precision,
                        walpha=wa, wbeta=wb)
    assert np.array_equal(plain.cand, wgt.cand)
    assert np.array_equal(plain.K, wgt.K)
    assert np.array_equal(plain.conv, wgt.conv)
    assert np.array_equal(plain.llr, wgt.llr)
    assert np.array_equal(plain.corr, wgt.corr)


def test_weighted_full_damping_keeps_prior():
    wl = WORKLOADS["bb72_L4_T20"]
    code = codes.bb72()
    ex, sx, bp, rows = _setup(code, wl, 50, 0.05)
    rng = np.random.default_rng(3)
    mu = rng.uniform(0.5, 4.0, size=(50, code.n))
    T = 6
    wa = rng.uniform(0.2, 1.5, size=(T, wl.L))
    res = oracle.decode(code.hz, bp, rows, sx, mu, T, rule=oracle.WNMS, fixed_T=True, want_llr=True,
                        walpha=wa, wbeta=np.ones((T, wl.L)))
    assert np.array_equal(res.llr, np.broadcast_to(mu[:, None, :], res.llr.shape))


def test_weighted_iteration_one_closed_form():
    """With uniform prior mu every v->c message of iteration 1 is mu, so every
    c->v message is (1 - beta_1) * alpha_1 * mu * (-1)^{s_j} and
    P^(1)_i = mu + (1 - beta_1) * alpha_1 * mu * sum over the augmented checks j of
    variable i of (-1)^{s_j}."""
    wl = WORKLOADS["bb72_L4_T20"]
    code = codes.bb72()
    ex, sx, bp, rows = _setup(code, wl, 40, 0.05)
    mu0 = 2.25
    a1 = np.array([[0.9, 0.6, 1.3, 0.75]])
    b1 = np.array([[0.0, 0.4, 0.25, 0.9]])
    res = oracle.decode(code.hz, bp, rows, sx, np.full(code.n, mu0), 1, rule=oracle.WNMS, fixed_T=True,
                        want_llr=True, walpha=a1, wbeta=b1)
    s = oracle.unpack(sx, code.hz.shape[0]).astype(np.int64)
    for l in range(wl.L):
        app = rows[bp[l]:bp[l + 1]]
        haug = np.vstack([code.hz, code.hz[app]]).astype(np.int64)
        saug = np.concatenate([s, s[:, app]], axis=1)
        signed = (1 - 2 * saug) @ haug
        expect = mu0 + (1 - b1[0, l]) * (a1[0, l] * mu0) * signed
        np.testing.assert_allclose(res.llr[:, l, :], expect, rtol=0, atol=1e-12)


def test_weighted_two_iterations_path_graph():
    """Checks c0 = {v0, v1}, c1 = {v1, v2}, s = (0, 1), mu = (1, 2, 3),
    alpha = (0.8, 0.5), beta = (0.25, 0.5), so k_t = (1 - beta_t) alpha_t = (0.6, 0.25).
    Iteration 1: r(c0->v0) = 0.6*2 = 1.2, r(c0->v1) = 0.6*1 = 0.6,
                 r(c1->v1) = -0.6*3 = -1.8, r(c1->v2) = -0.6*2 = -1.2;
                 q(v0->c0) = 1, q(v1->c0) = 2 - 1.8 = 0.2, q(v1->c1) = 2 + 0.6 = 2.6,
                 q(v2->c1) = 3.
    Iteration 2: r(c0->v0) = 0.25*0.2 + 0.5*1.2 = 0.65,
                 r(c0->v1) = 0.25*1 + 0.5*0.6 = 0.55,
                 r(c1->v1) = -0.25*3 + 0.5*(-1.8) = -1.65,
                 r(c1->v2) = -0.25*2.6 + 0.5*(-1.2) = -1.25.
    P^(2) = (1 + 0.65, 2 + 0.55 - 1.65, 3 - 1.25) = (1.65, 0.9, 1.75)."""
    h = np.array([[1, 1, 0], [0, 1, 1]], np.uint8)
    syn = oracle.pack(np.array([[0, 1]], np.uint8))
    res = oracle.decode(h, np.array([0, 0], np.int32), np.zeros(0, np.int32), syn, np.array([1.0, 2.0, 3.0]), 2,
                        rule=oracle.WNMS, fixed_T=True, want_llr=True,
                        walpha=np.array([[0.8], [0.5]]), wbeta=np.array([[0.25], [0.5]]))
    np.testing.assert_allclose(res.llr[0, 0], [1.65, 0.9, 1.75], rtol=0, atol=1e-12)


def test_weighted_rejects_serial_and_missing_weights():
    h = np.array([[1, 1, 0], [0, 1, 1]], np.uint8)
    syn = oracle.pack(np.array([[0, 1]], np.uint8))
    bp, rows = np.array([0, 0], np.int32), np.zeros(0, np.int32)
    with pytest.raises(oracle.OracleError):
        oracle.decode(h, bp, rows, syn, np.ones(3), 2, schedule=oracle.LAYERED, rule=oracle.WNMS,
                      walpha=np.ones((2, 1)), wbeta=np.zeros((2, 1)))


# ------------------------------------------------------------------ PyTorch reference

def _weights(T, L, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.6, 1.1, size=(T, L)), rng.uniform(0.0, 0.4, size=(T, L))


@pytest.mark.parametrize("precision,dtype", [("f64", torch.float64), ("f32", torch.float32)])
def test_torch_reference_forward_equals_oracle(precision, dtype):
    wl = WORKLOADS["bb72_L4_T20"]
    code = codes.bb72()
    shots, T = 60, 12
    ex, sx, bp, rows = _setup(code, wl, shots, 0.06)
    wa, wb = _weights(T, wl.L, 11)
    mu = np.full(code.n, oracle.prior_llr(0.06))
    res = oracle.decode(code.hz, bp, rows, sx, mu, T, rule=oracle.WNMS, fixed_T=True, want_llr=True,
                        precision=precision, walpha=wa, wbeta=wb)
    s = oracle.unpack(sx, code.hz.shape[0])
    cast = np.float32 if dtype == torch.float32 else np.float64
    for l in range(wl.L):
        rep = ref.Rep(code.hz, rows[bp[l]:bp[l + 1]])
        P = ref.forward(rep, s, torch.tensor(mu.astype(cast)), torch.tensor(wa[:, l].astype(cast)),
                        torch.tensor(wb[:, l].astype(cast)), T)
        got = P.numpy().astype(np.float64)
        assert np.array_equal(got, res.llr[:, l, :]), f"basis {l}"


def _oracle_loss(code, bp, rows, sx, mu, target, T, wa, wb, mask):
    res = oracle.decode(code.hz, bp, rows, sx, mu, T, rule=oracle.WNMS, fixed_T=True, want_llr=True,
                        walpha=wa, wbeta=wb)
    P = res.llr
    x = -P
    bce = np.maximum(x, 0) - x * target + np.log1p(np.exp(-np.abs(x)))
    return float((bce * mask[:, :, None]).sum() / (mask.sum() * code.n)), res


def test_torch_reference_gradient_matches_finite_differences():
    """Autograd of the float64 reference against central differences (h = 1e-7) of
    the FP64 oracle's loss, over the instances whose trajectory stays at least 1e-4
    from every non-smooth point of the forward map.  Per-qubit priors are drawn at
    random so that no two messages coincide by symmetry."""
    wl = WORKLOADS["bb72_L4_T20"]
    code = codes.bb72()
    shots, T, L = 8, 6, wl.L
    ex, sx, bp, rows = _setup(code, wl, shots, 0.08, seed=5)
    wa, wb = _weights(T, L, 17)
    mu = np.random.default_rng(23).uniform(1.0, 4.0, size=(shots, code.n))
    target = oracle.unpack(ex, code.n)[:, None, :].astype(np.float64) * np.ones((1, L, 1))
    _, res0 = _oracle_loss(code, bp, rows, sx, mu, target, T, wa, wb, np.ones((shots, L)))
    mask = (res0.margin[..., 0] > 1e-4).astype(np.float64)
    assert mask.sum() >= shots * L // 2, "too few smooth instances for the check"
    # autograd of the reference
    s = oracle.unpack(sx, code.hz.shape[0])
    A = torch.tensor(wa, requires_grad=True)
    B = torch.tensor(wb, requires_grad=True)
    total = 0
    weight = torch.tensor(mask / (mask.sum() * code.n))
    for l in range(L):
        rep = ref.Rep(code.hz, rows[bp[l]:bp[l + 1]])
        P = ref.forward(rep, s, torch.tensor(mu), A[:, l], B[:, l], T)
        total = total + ref.loss_fn(P, torch.tensor(target[:, l, :]),
                                    weight[:, l, None].expand(shots, code.n))
    total.backward()
    ga, gb = A.grad.numpy(), B.grad.numpy()
    h = 1e-7
    for which, g in (("alpha", ga), ("beta", gb)):
        fd = np.zeros_like(g)
        for t in range(T):
            for l in range(L):
                pa, pb = wa.copy(), wb.copy()
                (pa if which == "alpha" else pb)[t, l] += h
                lp, _ = _oracle_loss(code, bp, rows, sx, mu, target, T, pa, pb, mask)
                (pa if which == "alpha" else pb)[t, l] -= 2 * h
                lm, _ = _oracle_loss(code, bp, rows, sx, mu, target, T, pa, pb, mask)
                fd[t, l] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8, err_msg=which)
    assert np.abs(ga).max() > 1e-4 and np.abs(gb).max() > 1e-4
