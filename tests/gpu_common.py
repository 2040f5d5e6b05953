"""Helpers shared by the GPU parity tests (inputs from ``workloads``, expected
values from ``oracle``; nothing expected ever comes from the HIP path)."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def device():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda:0")


def api():
    from paper_1312_1869_amd import api as a  # raises if liblrinv.so is missing

    return a


def note(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def omega_pair(w: W.Workload, prec: str, dev, n: int | None = None, d: int | None = None):
    """(oracle omega dict, device Omega) for a workload."""
    a = api()
    n = w.n if n is None else n
    d = w.d if d is None else d
    if w.omega == "srht":
        signs, cols = W.srht_draw(w, n, d)
        return {"kind": "srht", "signs": signs, "cols": cols}, a.Omega.srht(signs, cols, dev)
    om_t = W.gauss_omega(w, n, d, round_bf16=(prec in ("bf16", "bf16x2")))
    return {"kind": "gauss", "omega_t": om_t}, a.Omega.gauss(om_t, prec, dev)


def hyper(w: W.Workload):
    return api().Hyper(w.kernel, w.ell, w.s)


def to_dev(x: np.ndarray, dtype, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=dev, dtype=dtype)


def rel_max(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def qr_fp32(y):
    """Precision model of a float32 QR: LAPACK's float32 Householder QR
    (scipy) of float32(y), signs fixed so diag(R) >= 0, promoted to float64.
    Used only to measure how strongly the float64 method reacts to the
    rounding a float32 path introduces; it is not a step of the method."""
    import scipy.linalg as sla

    q, r = sla.qr(np.asarray(y, dtype=np.float32), mode="economic")
    sg = np.where(np.diag(r) < 0, -1.0, 1.0)
    return q.astype(np.float64) * sg[None, :], r.astype(np.float64) * sg[:, None]


def qr_fp64(y):
    """LAPACK's float64 Householder QR (numpy) with diag(R) >= 0: a fast
    float64 QR for sampling how the method reacts to perturbed sketches."""
    q, r = np.linalg.qr(np.asarray(y, dtype=np.float64))
    sg = np.where(np.diag(r) < 0, -1.0, 1.0)
    return q * sg[None, :], r * sg[:, None]


def fl32(a):
    return np.asarray(a).astype(np.float32).astype(np.float64)


def log2n(n: int) -> float:
    return max(1.0, math.log2(n))
