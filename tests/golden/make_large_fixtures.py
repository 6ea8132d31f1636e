"""Writes tests/golden/large_forced.json: the oracle's results at the two
full-size lattices, at fixed (forced) iteration counts, as sampled entries
the GPU tests compare against.  Calls only oracle/ (and the seeded input
generators of workloads/); it takes about 20 minutes on one CPU core.

    python tests/golden/make_large_fixtures.py

Cases:
  * 24^3x48, the Gaussian source, N_s = 58 Neuberger poles, l = 2 with 2 and
    l = 6 with 1 forced outer iteration: y (double pass, all 58 shifts) and
    x_s of three shifts (single pass restricted to those shifts -- the seed
    iteration does not depend on the shifts, so those x_s are the full
    solve's), plus the stencil gamma5 D b;
  * 16^3x32, point sources 0 and 6 of the 12, N_s = 30, l = 4, with the
    per-(source, shift) forced freeze iterations FORCE below (3 to 5 outer
    iterations for source 0, 3 to 11 for source 6): y and x_s of three shifts
    (single pass).

Each stored vector is kept as: its 2-norm, 512 entries at seeded random
flat indices (complex as [re, im]) and its inner products with two seeded
Gaussian vectors.  Each case also records the oracle's own sensitivity: the
relative change of its y when b is perturbed by 1e-15 relative (seeded),
which sets the parity bound where it exceeds 1e-10 (l = 6: the MR normal
equations of six Krylov vectors amplify rounding), and for the 16^3x32
sources every shift's M_s.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import dirac as od  # noqa: E402
from oracle import krylov as ok  # noqa: E402
from oracle import pfe  # noqa: E402

NSAMPLE = 512
PROJ_SEEDS = (9101, 9102)


def force_16(nrhs, ns):
    """Forced freeze iterations of the 16^3x32 batch: shift s of source r
    stops after 3 + (s + r) mod (3 + r mod 7) outer iterations."""
    r = np.arange(nrhs)[:, None]
    s = np.arange(ns)[None, :]
    return (3 + (s + r) % (3 + r % 7)).astype(np.int32)


def perturbed(b, seed):
    rng = np.random.default_rng(seed)
    return b * (1 + 1e-15 * rng.standard_normal(b.shape))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sample_indices(n, seed):
    return np.sort(np.random.default_rng(seed).choice(n, NSAMPLE, replace=False))


def fingerprint(v, dims, idx):
    flat = v.reshape(-1)
    proj = []
    for sd in PROJ_SEEDS:
        z = wl.gaussian_source(dims, sd)[0].reshape(-1)
        c = complex(np.vdot(z, flat))
        proj.append([c.real, c.imag])
    return {"norm": float(np.linalg.norm(flat)), "samples": [[float(x.real), float(x.imag)] for x in flat[idx]],
            "proj": proj}


# the normalisation of A: any positive constant is a valid input and both
# sides receive the same one; 1/(1.01 * 36.5) bounds 1/lambda_max(D^+ D) of
# these fields (the power iteration at this size would take the oracle tens of
# minutes)
A_SCALE = 1.0 / (1.01 * 36.5)


def main():
    out = {"_source": "tests/golden/make_large_fixtures.py (oracle only)", "nsample": NSAMPLE,
           "proj_seeds": list(PROJ_SEEDS), "cases": {}}
    # ---- 24^3x48
    wk = wl.WORKLOADS["24x24x24x48"]
    t0 = time.time()
    op = od.Dirac(wk.links(), wk.dims, wk.mass, wk.mu, wk.bc_t)
    a = A_SCALE
    sig, w = pfe.neuberger(wk.n_shift)
    b = wk.sources()[0]
    n = b.size
    idx = sample_indices(n, 9001)
    out["cases"]["24x24x24x48 stencil"] = {"a_scale": a, "sample_seed": 9001,
                                          "g5_dw_b": fingerprint(od.g5(op.dw(b)), wk.dims, idx)}
    print(f"24^3x48 set-up and stencil {time.time() - t0:.0f} s", flush=True)
    amv = lambda v: op.a_op(v, a)
    for l, M in ((2, 2), (6, 1)):
        t0 = time.time()
        force = np.full(len(sig), M)
        y, info = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, M, 2, force_iters=force)
        yp = ok.mshift_bicgstabl(amv, perturbed(b, 9301), sig, w, l, wk.tol, M, 2, force_iters=force)[0]
        keep = [0, 29, 57]
        _, i1, X = ok.mshift_bicgstabl(amv, b, sig[keep], w[keep], l, wk.tol, M, 1,
                                       force_iters=force[keep])
        out["cases"][f"24x24x24x48 l={l} M={M}"] = {
            "a_scale": a, "l": l, "forced_outer": M, "sample_seed": 9001, "shifts_kept": keep,
            "status": int(info.status), "sensitivity": rel(yp, y), "y": fingerprint(y, wk.dims, idx),
            "x": [fingerprint(x, wk.dims, idx) for x in X]}
        print(f"24^3x48 l={l}: {time.time() - t0:.0f} s, sensitivity {rel(yp, y):.2e}", flush=True)
        del y, yp, X
    del op
    # ---- 16^3x32
    wk = wl.WORKLOADS["16x16x16x32"]
    t0 = time.time()
    op = od.Dirac(wk.links(), wk.dims, wk.mass, wk.mu, wk.bc_t)
    a = A_SCALE
    sig, w = pfe.neuberger(wk.n_shift)
    src = wl.point_sources(wk.dims)
    F = force_16(src.shape[0], len(sig))
    idx = sample_indices(src[0].size, 9002)
    amv = lambda v: op.a_op(v, a)
    for r in (0, 6):
        y, info, X = ok.mshift_bicgstabl(amv, src[r], sig, w, 4, wk.tol, int(F[r].max()), 1, force_iters=F[r])
        yp = ok.mshift_bicgstabl(amv, perturbed(src[r], 9302 + r), sig, w, 4, wk.tol, int(F[r].max()), 2,
                                 force_iters=F[r])[0]
        keep = [0, 15, 29]
        out["cases"][f"16x16x16x32 source {r}"] = {
            "a_scale": a, "l": 4, "source": r, "force": F[r].tolist(), "sample_seed": 9002,
            "shifts_kept": keep, "status": int(info.status), "outer": int(info.outer),
            "shift_iters": info.shift_iters.tolist(), "sensitivity": rel(yp, y),
            "y": fingerprint(y, wk.dims, idx), "x": [fingerprint(X[s], wk.dims, idx) for s in keep]}
        print(f"16^3x32 source {r}: {time.time() - t0:.0f} s, sensitivity {rel(yp, y):.2e}", flush=True)
        del y, yp, X
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_forced.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}")


if __name__ == "__main__":
    main()
