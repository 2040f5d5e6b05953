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
    om_t = W.gauss_omega(w, n, d, round_bf16=(prec == "bf16"))
    return {"kind": "gauss", "omega_t": om_t}, a.Omega.gauss(om_t, prec, dev)


def hyper(w: W.Workload):
    return api().Hyper(w.kernel, w.ell, w.s)


def to_dev(x: np.ndarray, dtype, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device=dev, dtype=dtype)


def rel_max(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def log2n(n: int) -> float:
    return max(1.0, math.log2(n))
