"""GPU parity of lr_tsqr against the oracle's binary-tree Householder QR.

R with diag(R) >= 0 is unique for full-column-rank Y, so on well-conditioned
inputs R and Q are compared entry by entry; its perturbation is of order
cond(Y) * sqrt(n d) * u. On ill-conditioned kernel sketches (where only the
leading part of R is determined) the test checks what holds at any
conditioning: Q^T Q = I, Q R = Y, R upper triangular with diag >= 0.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import qr as oqr

from gpu_common import U32, U64, api, device, hyper, note, omega_pair, to_dev, torch

pytestmark = pytest.mark.gpu


def _gauss_y(n, d, seed, decay=2.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, d)) @ np.diag(np.logspace(0, -math.log10(decay), d))


def _run(y, leaf, prec, dev):
    a = api()
    dt = torch.float64 if prec == "f64" else torch.float32
    Y = to_dev(y, dt, dev)
    note(f"tsqr n={y.shape[0]} d={y.shape[1]} leaf={leaf} prec={prec}")
    Q, R = a.tsqr(Y, leaf, prec)
    torch.cuda.synchronize()
    return Y, Q, R


def _props(Y, Q, R):
    q = Q.double()
    d = q.shape[1]
    orth = (q.T @ q - torch.eye(d, dtype=torch.float64, device=q.device)).abs().max().item()
    back = ((q @ R - Y.double()).norm() / Y.double().norm()).item()
    r = R.cpu().numpy()
    return orth, back, r


@pytest.mark.parametrize("n,d,leaf", [(2048, 64, 128), (1000, 20, 96), (4096, 48, 4096), (777, 7, 7),
                                      (512, 128, 128)])
def test_tsqr_f64_matches_oracle(n, d, leaf):
    dev = device()
    y = _gauss_y(n, d, n + d)
    Y, Q, R = _run(y, leaf, "f64", dev)
    qo, ro = oqr.tsqr(y, leaf)
    orth, back, r = _props(Y, Q, R)
    note(f"  orth {orth:.2e} back {back:.2e}")
    assert np.all(np.tril(r, -1) == 0.0) and np.all(np.diag(r) >= 0)
    assert orth <= 50 * math.sqrt(n) * U64 and back <= 50 * math.sqrt(n) * U64
    np.testing.assert_allclose(r, ro, rtol=0, atol=1e-12 * np.abs(ro).max())
    np.testing.assert_allclose(Q.cpu().numpy(), qo, rtol=0, atol=1e-11)


@pytest.mark.parametrize("n,d,leaf", [(8492, 200, 1024), (16384, 256, 4096), (4096, 64, 512)])
def test_tsqr_f32_matches_oracle(n, d, leaf):
    dev = device()
    y = _gauss_y(n, d, 7 * n + d)
    y32 = y.astype(np.float32)
    Y, Q, R = _run(y32, leaf, "f32", dev)
    qo, ro = oqr.tsqr(y32.astype(np.float64), leaf)
    orth, back, r = _props(Y, Q, R)
    err_r = np.abs(r - ro).max() / np.abs(ro).max()
    err_q = np.abs(Q.double().cpu().numpy() - qo).max()
    note(f"  orth {orth:.2e} back {back:.2e} R err {err_r:.2e} Q err {err_q:.2e}")
    tol = 20 * math.sqrt(n) * U32
    assert np.all(np.tril(r, -1) == 0.0) and np.all(np.diag(r) >= 0)
    assert orth <= tol and back <= tol and err_r <= 4 * tol and err_q <= 4 * tol


def test_tsqr_tree_shape_invariance_f64():
    dev = device()
    y = _gauss_y(8192, 96, 5)
    rs = [_run(y, leaf, "f64", dev)[2].cpu().numpy() for leaf in (8192, 2048, 1000, 128)]
    for r in rs[1:]:
        np.testing.assert_allclose(r, rs[0], rtol=0, atol=1e-12 * np.abs(rs[0]).max())


@pytest.mark.parametrize("name,prec", [("C1", "f64"), ("C2", "f32"), ("C3", "bf16")])
def test_tsqr_kernel_sketch_full_size_properties(name, prec):
    dev = device()
    a = api()
    w = W.WORKLOADS[name]
    x = W.points(w)
    _, om = omega_pair(w, prec, dev)
    X = to_dev(x, torch.float32, dev)
    note(f"tsqr on sketch {name} prec={prec}")
    Y, _ = a.sketch(X, hyper(w), om, prec)
    rp = "f32" if prec == "bf16" else prec
    Q, R = a.tsqr(Y, w.leaf_rows, rp)
    torch.cuda.synchronize()
    orth, back, r = _props(Y, Q, R)
    u = U64 if prec == "f64" else U32
    note(f"  orth {orth:.2e} back {back:.2e}")
    assert np.all(np.tril(r, -1) == 0.0) and np.all(np.diag(r) >= 0)
    assert orth <= 50 * math.sqrt(w.n) * u
    assert back <= 50 * math.sqrt(w.n) * u


def _unique_qr(y):
    """QR of a full-rank y with R's diagonal made positive: then Q and R are
    unique, so any correct algorithm (here LAPACK's) gives the same factors."""
    q, r = np.linalg.qr(y)
    sg = np.where(np.diag(r) < 0, -1.0, 1.0)
    return q * sg[None, :], r * sg[:, None]


@pytest.mark.parametrize("prec,n,d,leaf", [("f64", 4096, 1024, 2048), ("f32", 6144, 1024, 1536)])
def test_tsqr_largest_d_matches_unique_qr(prec, n, d, leaf):
    """d = 1024, the largest rank the boundary takes (tree panels with several
    rows per thread). The pin is the unique positive-diagonal QR."""
    dev = device()
    y = _gauss_y(n, d, 11 * n + d)
    if prec == "f32":
        y = y.astype(np.float32)
    Y, Q, R = _run(y, leaf, prec, dev)
    qo, ro = _unique_qr(np.asarray(y, dtype=np.float64))
    orth, back, r = _props(Y, Q, R)
    u = U64 if prec == "f64" else U32
    err_r = np.abs(r - ro).max() / np.abs(ro).max()
    err_q = np.abs(Q.double().cpu().numpy() - qo).max()
    note(f"  orth {orth:.2e} back {back:.2e} R err {err_r:.2e} Q err {err_q:.2e}")
    assert np.all(np.tril(r, -1) == 0.0) and np.all(np.diag(r) >= 0)
    if prec == "f64":
        assert orth <= 50 * math.sqrt(n) * u and back <= 50 * math.sqrt(n) * u
        assert err_r <= 1e-12 and err_q <= 1e-11
    else:
        tol = 20 * math.sqrt(n) * u
        assert orth <= tol and back <= tol and err_r <= 4 * tol and err_q <= 4 * tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("group", [1, 2, 4, 8])
def test_tsqr_tree_groups_match_oracle(prec, group):
    """lr_tsqr_tree: groups of blocks run in sequence (Eq. 5) under the binary
    tree, against the oracle's grouped scheme (group = 1: the binary tree;
    group = 8 = the number of blocks: fully sequential), with and without Q."""
    dev = device()
    a = api()
    n, d, leaf = 8 * 512, 64, 512
    y = _gauss_y(n, d, 31 * group)
    if prec == "f32":
        y = y.astype(np.float32).astype(np.float64)
    dt = torch.float64 if prec == "f64" else torch.float32
    Y = to_dev(y, dt, dev)
    note(f"tsqr tree n={n} d={d} leaf={leaf} group={group} prec={prec}")
    Q, R = a.tsqr_tree(Y, leaf, prec, group=group)
    _, R_only = a.tsqr_tree(Y, leaf, prec, group=group, want_q=False)
    torch.cuda.synchronize()
    qo, ro = oqr.tsqr_grouped(y, leaf, group)
    orth, back, r = _props(Y, Q, R)
    u = U64 if prec == "f64" else U32
    err_r = np.abs(r - ro).max() / np.abs(ro).max()
    err_q = np.abs(Q.double().cpu().numpy() - qo).max()
    note(f"  R rel {err_r:.2e} Q {err_q:.2e} orth {orth:.2e} back {back:.2e}")
    assert np.all(np.tril(r, -1) == 0.0) and np.all(np.diag(r) >= 0)
    assert orth <= 50 * math.sqrt(n) * u and back <= 50 * math.sqrt(n) * u
    assert torch.equal(R, R_only)  # the same factorisation, Q never formed
    if prec == "f64":
        assert err_r <= 1e-12 and err_q <= 1e-11
    else:
        assert err_r <= 80 * math.sqrt(n) * u and err_q <= 80 * math.sqrt(n) * u
