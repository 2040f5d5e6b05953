"""GPU parity of the structured Omega written out by lr_structured_omega (the
discrete cosine and Hartley forms of Def. 1, Sec. 3.2, and Walsh-Hadamard),
and of the whole path run with it, against the oracle (oracle.transforms).

Entries: the GPU and the oracle each evaluate T[j, p] in float64 from the
closed form with the angle reduced exactly in integers, so their float64
values agree to a few units of the last place; the float32 and bf16 entries
are each side's rounding (nearest even) of its own float64 value, so they are
equal except where a float64 value lies within those few ulps of a rounding
midpoint (a vanishing fraction, bounded below). The path: sketch on the dense
matrix cores, TSQR and the Woodbury solve against the oracle's fast-transform
forms (scipy.fft), for n that is not a power of two.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import grad as og, kernels, sketch as osk, srht as osr, transforms as otr

from gpu_common import U32, U64, api, device, hyper, note, rel_max, to_dev, torch
from test_gpu_sketch import _bf16_ambiguity, _scale_dense

pytestmark = pytest.mark.gpu


def _draw(w, n, d):
    signs, cols = W.srht_draw(w, n, d)
    return signs, cols


def _oracle_omega_t(transform, signs, cols):
    n = signs.shape[0]
    if transform == "wht":
        return osr.entries(signs, cols, np.arange(n)).T
    return otr.omega_entries(transform, signs, cols, np.arange(n)).T


def _omega_dict(transform, signs, cols):
    return {"kind": "srht" if transform == "wht" else transform, "signs": signs, "cols": cols}


@pytest.mark.parametrize("transform,n", [("dct", 3000), ("dht", 3000), ("dct", 65536 + 40), ("dht", 1), ("wht", 4096)])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_structured_omega_entries(transform, n, prec):
    dev = device()
    a = api()
    w = W.WORKLOADS["C2"]
    d = min(96, n)
    signs, cols = _draw(w, n, d)
    note(f"structured omega {transform} n={n} d={d} prec={prec}")
    om = a.Omega.structured(transform, signs, cols, prec, dev)
    torch.cuda.synchronize()
    g = om.dense_t.float().double().cpu().numpy() if prec == "bf16" else om.dense_t.double().cpu().numpy()
    assert np.all(g[:, n:] == 0.0)
    g = g[:, :n]
    ref = _oracle_omega_t(transform, signs, cols)
    amax = math.sqrt(2.0 / n)
    if prec == "f64":
        err = np.abs(g - ref).max()
        note(f"  max |diff| {err:.2e} (entries up to {amax:.2e})")
        assert err <= 16 * U64 * amax
    else:
        r = ref.astype(np.float32).astype(np.float64) if prec == "f32" else osk.round_to_bf16(ref)
        ulp = (2.0 ** -23 if prec == "f32" else 2.0 ** -7) * np.exp2(np.floor(np.log2(np.maximum(np.abs(r), 1e-300))))
        diff = np.abs(g - r)
        frac = float(np.mean(diff > 0))
        note(f"  entries differing from the oracle's rounding: {frac:.2e} (at most one unit)")
        assert np.all(diff <= ulp) and frac <= 1e-4
    # the columns are orthonormal (to the output precision)
    gram = g @ g.T
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 0.05}[prec]
    assert np.abs(gram - np.eye(d)).max() <= tol


@pytest.mark.parametrize("transform", ["dct", "dht"])
def test_structured_forward_fp64(transform):
    """sketch -> TSQR -> Woodbury solve in FP64 with a cosine / Hartley Omega
    (n = 3000, not a power of two) against the oracle's fast-transform path."""
    dev = device()
    a = api()
    w = W.small(W.WORKLOADS["C2"], 3000, d=64, leaf_rows=1000, m=4)
    x = W.points(w)
    A = W.rhs(w)
    signs, cols = _draw(w, w.n, w.d)
    om = a.Omega.structured(transform, signs, cols, "f64", dev)
    note(f"structured forward {transform} fp64 n={w.n} d={w.d}")
    fw = a.forward(to_dev(x, torch.float32, dev), hyper(w), om, "f64", w.sigma2, to_dev(A, torch.float64, dev),
                   w.leaf_rows)
    torch.cuda.synchronize()
    ref = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, _omega_dict(transform, signs, cols), A, w.leaf_rows)
    assert int(fw.sol.info.item()) == 0 and ref["info"] == 0
    ex = rel_max(fw.sol.X.cpu().numpy(), ref["X"])
    el = abs(fw.sol.logdet.item() - ref["logdet"]) / abs(ref["logdet"])
    ey = np.abs(fw.Y.cpu().numpy() - ref["Y"]).max() / np.abs(ref["Y"]).max()
    note(f"  Y rel {ey:.2e} X rel {ex:.2e} logdet rel {el:.2e}")
    assert ey <= 1e-12 and ex <= 1e-10 and el <= 1e-10


@pytest.mark.parametrize("transform", ["dct", "dht"])
def test_structured_sketch_f32_and_bf16(transform):
    """The float32 and bf16 sketches with a written-out cosine / Hartley Omega:
    float32 within (4 sqrt(n) + 16) u32 of sum_j |K_ij| |Omega_jk|; bf16
    against the oracle with bf16-rounded K entries and the oracle's own bf16
    Omega, up to the midpoint ambiguity of the K rounding."""
    dev = device()
    a = api()
    w = W.small(W.WORKLOADS["C2"], 5000, d=128)
    x = W.points(w)
    signs, cols = _draw(w, w.n, w.d)
    X = to_dev(x, torch.float32, dev)
    om_t = _oracle_omega_t(transform, signs, cols)
    rows = np.arange(w.n)
    for prec in ("f32", "bf16"):
        note(f"structured sketch {transform} {prec} n={w.n} d={w.d}")
        om = a.Omega.structured(transform, signs, cols, prec, dev)
        Y, _ = a.sketch(X, hyper(w), om, prec)
        torch.cuda.synchronize()
        y = Y.double().cpu().numpy()
        if prec == "f32":
            om32 = om_t.astype(np.float32).astype(np.float64)
            ref = osk.sketch(x, w.kernel, w.ell, w.s, {"kind": "gauss", "omega_t": om32})
            sc = _scale_dense(x, rows, w, om32)
            err = (np.abs(y - ref) / sc).max()
            note(f"  max err / scale {err:.2e}")
            assert err <= (4 * math.sqrt(w.n) + 16) * U32
        else:
            omb = osk.round_to_bf16(om_t)
            ref = osk.sketch(x, w.kernel, w.ell, w.s, {"kind": "gauss", "omega_t": omb}, k_round="bf16")
            sc = _scale_dense(x, rows, w, omb)
            amb = _bf16_ambiguity(x, rows, w, omb)
            # an Omega entry whose float64 value sits on a bf16 midpoint may round
            # the other way on the GPU (checked rare above): allow its difference
            dom = np.abs(om.dense_t.float().double().cpu().numpy()[:, :w.n] - omb)
            if dom.any():
                amb = amb + np.abs(kernels.kernel_matrix(w.kernel, x, x, w.ell, w.s)) @ dom.T
            excess = np.maximum(np.abs(y - ref) - amb, 0.0) / sc
            note(f"  max excess over the rounding ambiguity / scale {excess.max():.2e}")
            assert excess.max() <= 4 * math.sqrt(w.n) * U32


@pytest.mark.parametrize("transform", ["dct", "dht"])
def test_structured_loglik_gradient_fp64(transform):
    """The log-likelihood adjoint in FP64 with a cosine / Hartley Omega against
    the oracle's gradient formulas (fast-transform Omega^T products)."""
    dev = device()
    a = api()
    w = W.small(W.WORKLOADS["C4"], 2500, d=48, leaf_rows=500)
    x = W.points(w)
    yv = W.gp_targets(w, x)
    signs, cols = _draw(w, w.n, w.d)
    om = a.Omega.structured(transform, signs, cols, "f64", dev)
    X = to_dev(x, torch.float32, dev)
    yd = to_dev(yv.reshape(-1, 1), torch.float64, dev)
    note(f"structured loglik gradient {transform} fp64 n={w.n} d={w.d}")
    fw = a.forward(X, hyper(w), om, "f64", w.sigma2, yd, w.leaf_rows, want_yprime=True)
    dth, _ = a.backward(X, hyper(w), om, "f64", fw.sol, fw.Q, w.sigma2, 0, yd, Yprime=fw.Yprime, R=fw.R)
    torch.cuda.synchronize()
    omd = _omega_dict(transform, signs, cols)
    f = og.forward(x, w.kernel, w.ell, w.s, w.sigma2, omd, yv.reshape(-1, 1), w.leaf_rows)
    g_ref, parts = og.grad_loglik(x, w.kernel, w.ell, w.s, w.sigma2, omd, f["Q"], f, yv, parts=True)
    g = dth.cpu().numpy()
    note(f"  grad {g} oracle {g_ref}")
    assert np.all(np.abs(g - g_ref) <= 1e-9 * parts + 1e-9 * np.abs(g_ref))
