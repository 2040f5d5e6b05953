"""Write tests/golden/c4_oracle_reference.txt: the FP64 oracle's log-likelihood
workload (n = 32768 uniform points in [0,1]^2, squared-exponential kernel
s = 1.5, ell = 0.25, sigma2 = 1e-2, SRHT Omega with d = 256, 8 leaves of 4096
rows, targets from the seeded GP draw of ``workloads.gp_targets``).

Recorded: log|K~|, the log-likelihood and its gradient in (log ell, log s,
log sigma2) from the oracle alone; the same quantities from the oracle fed
the float32 rounding of its own sketches Y and Y' (every stage after the
sketch still in float64); and from a precision model of a float32 path:
those rounded sketches, a float32 Householder QR of Y (LAPACK's sgeqrf via
scipy, signs fixed so diag(R) >= 0), then the float64 core and gradient. The
last two sets measure how strongly the float64 method itself reacts to
float32 rounding of the sketch and of its QR; a run with LAPACK's float64
QR in place of the oracle's own tree QR measures how much two float64 QRs of
the same sketch move the result. The same oracle and model are
also run with the stabilising shift nu = 1e-3 (Y = (K_f + nu I) Omega), under
which the float32 model's core stays positive definite. Nothing here comes
from the HIP library.

Run from the repository root: ``python tests/golden/make_c4_reference.py``
(about five minutes on eight cores).
"""
from __future__ import annotations

import os
import sys

import numpy as np
import scipy.linalg as sla

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import grad as og, lowrank as ol, qr as oqr, sketch as osk  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_oracle_reference.txt")


def qr_fp32(y):
    """float32 Householder QR (LAPACK) of float32 y, diag(R) >= 0, promoted."""
    q, r = sla.qr(np.asarray(y, dtype=np.float32), mode="economic")
    sg = np.where(np.diag(r) < 0, -1.0, 1.0)
    return q.astype(np.float64) * sg[None, :], r.astype(np.float64) * sg[:, None]


def qr_fp64_lapack(y):
    """LAPACK's float64 Householder QR (numpy), diag(R) >= 0."""
    q, r = np.linalg.qr(np.asarray(y, dtype=np.float64))
    sg = np.where(np.diag(r) < 0, -1.0, 1.0)
    return q * sg[None, :], r * sg[:, None]


def run(x, w, om, yv, y, yp, qr32=False, nu=0.0, lapack64=False):
    if lapack64:
        q, r = qr_fp64_lapack(y)
    else:
        q, r = qr_fp32(y) if qr32 else oqr.tsqr(y, w.leaf_rows)
    core = ol.solve(q, r, om, w.sigma2, yv.reshape(-1, 1), nu)
    if core["info"] != 0:
        return core["info"], None, None, np.full(3, np.nan)
    ll = ol.loglik(yv, core["X"][:, 0], core["logdet"])
    g = og.grad_loglik(x, w.kernel, w.ell, w.s, w.sigma2, om, q, core, yv, yprime=yp, nu=nu, r=r)
    return 0, core["logdet"], ll, g


# the stabilising shift used for the float32 path (a tenth of the nugget)
NU = 1e-3


def main() -> None:
    w = W.WORKLOADS["C4"]
    x = W.points(w)
    yv = W.gp_targets(w, x)
    signs, cols = W.srht_draw(w)
    om = {"kind": "srht", "signs": signs, "cols": cols}
    y = osk.sketch(x, w.kernel, w.ell, w.s, om)
    yp = osk.sketch(x, w.kernel, w.ell, w.s, om, deriv=True)
    y32, yp32 = fl32(y), fl32(yp)
    rows = {}
    rows[""] = run(x, w, om, yv, y, yp)
    rows["_f64lapack"] = run(x, w, om, yv, y, yp, lapack64=True)
    rows["_fl32sketch"] = run(x, w, om, yv, y32, yp32)
    rows["_fp32model"] = run(x, w, om, yv, y32, yp32, qr32=True)
    ynu = y + NU * osk.omega_rows(om, np.arange(w.n))
    rows["_nu"] = run(x, w, om, yv, ynu, yp, nu=NU)
    rows["_nu_fp32model"] = run(x, w, om, yv, fl32(ynu), yp32, qr32=True, nu=NU)
    lines = [
        "# FP64 oracle at the full log-likelihood workload (n=32768, D=2, SE s=1.5 ell=0.25",
        "# sigma2=1e-2, SRHT d=256, 8 leaves of 4096 rows, GP targets from workloads.gp_targets).",
        "# Written by tests/golden/make_c4_reference.py (oracle and workloads only).",
        "# name value. Suffixes: (none) the oracle, shift nu = 0; _f64lapack the same with LAPACK's float64",
        "# QR in place of the oracle's tree QR; _fl32sketch fed fl32(Y), fl32(Y');",
        "# _fp32model fed fl32(Y), fl32(Y') and a float32 LAPACK QR of fl32(Y); _nu the oracle with the",
        f"# shift nu = {NU!r}; _nu_fp32model its float32 model. info != 0: the Cholesky of S failed.",
        f"nu {float(NU)!r}",
    ]
    for suf, (info, ld, ll, g) in rows.items():
        lines.append(f"info{suf} {int(info)}")
        if info == 0:
            lines += [f"logdet{suf} {float(ld)!r}", f"loglik{suf} {float(ll)!r}", f"grad_logell{suf} {float(g[0])!r}",
                      f"grad_logs{suf} {float(g[1])!r}", f"grad_logsigma2{suf} {float(g[2])!r}"]
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def fl32(a):
    return np.asarray(a).astype(np.float32).astype(np.float64)


if __name__ == "__main__":
    main()
