"""Oracle parity at the two full-size lattices, at fixed (forced) iteration
counts, against the oracle's sampled results in tests/golden/large_forced.json
(written by tests/golden/make_large_fixtures.py, which calls only the oracle):

  * 24^3x48, one Gaussian source, N_s = 58, l = 2 (2 outer iterations) and
    l = 6 (1): y of the per-step and the deferred single pass, the double and
    the pseudo-double pass, x_s of three shifts, and the stencil gamma5 D b;
  * 16^3x32, the 12 point sources in one batch, N_s = 30, l = 4, with the
    freeze iteration forced per (source, shift) between 3 and 11: shifts
    freeze inside the batch at different iterations, source 0 stops after 5
    outer iterations while source 6 runs 11 (past the pseudo-double pass's
    first 8-iteration storage chunk); sources 0 and 6 are compared.

A stored vector is compared through its 512 sampled entries (their relative
2-norm error estimates the whole vector's), its norm and two inner products
with seeded Gaussian vectors.  Bound: 1e-10 relative in FP64, or 30x the
oracle's own sensitivity (its y's change under a 1e-15 relative perturbation
of b, recorded with the fixture) where that is larger -- at l = 6 the MR
normal equations of six Krylov vectors amplify rounding; the stencil 1e-14.
Shifts freeze at the forced iteration unless their |zeta psi| outgrows 1e300
first (then they stop as converged): M_s is compared with the oracle's.
"""
import importlib.util
import json
import os

import numpy as np
import pytest

import workloads as wl
from tests.helpers import cuda, log

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
FIX = os.path.join(HERE, "golden", "large_forced.json")


def fixture():
    with open(FIX) as f:
        return json.load(f)


def force_16(nrhs, ns):
    spec = importlib.util.spec_from_file_location("mlf", os.path.join(HERE, "golden", "make_large_fixtures.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.force_16(nrhs, ns)


class Fingerprint:
    def __init__(self, fx, dims, seed):
        self.fx = fx
        n = 12 * wl.volume(dims)
        self.idx = np.sort(np.random.default_rng(seed).choice(n, fx["nsample"], replace=False))
        self.z = [wl.gaussian_source(dims, sd)[0].reshape(-1) for sd in fx["proj_seeds"]]

    def errors(self, v, ref):
        """(sampled relative error, norm error, largest projection error) of
        the device vector v (complex128 torch tensor) against a stored one."""
        import torch
        flat = v.reshape(-1)
        samp = flat[torch.from_numpy(self.idx).to(flat.device)].cpu().numpy()
        rs = np.array([complex(a, b) for a, b in ref["samples"]])
        nrm = float(torch.linalg.vector_norm(flat))
        e_s = float(np.linalg.norm(samp - rs) / np.linalg.norm(rs))
        e_n = abs(nrm - ref["norm"]) / ref["norm"]
        e_p = 0.0
        for z, (pr, pi) in zip(self.z, ref["proj"]):
            c = complex(torch.vdot(torch.from_numpy(z).to(flat.device), flat))
            e_p = max(e_p, abs(c - complex(pr, pi)) / (np.linalg.norm(z) * ref["norm"]))
        return e_s, e_n, e_p


def bound_of(case):
    return max(1e-10, 30 * case["sensitivity"])


def check(name, errs, bound):
    e_s, e_n, e_p = errs
    log(f"  {name}: sampled {e_s:.2e}, norm {e_n:.2e}, projection {e_p:.2e}")
    assert e_s <= bound and e_n <= bound and e_p <= bound, name


FORMS = [("pass 1", 1, 0, True), ("pass 1 deferred", 1, "DEFERRED", True), ("pass 2", 2, 0, False),
         ("pass 3", 3, 0, False), ("pass 2 seed basis", 2, "SEED_BASIS", False),
         ("pass 3 seed basis", 3, "SEED_BASIS", False)]


@pytest.fixture(scope="module")
def big():
    import torch
    from paper_1010_2592_amd import msb
    wk = wl.WORKLOADS["24x24x24x48"]
    log("24x24x24x48: inputs")
    U = cuda(wk.links())
    b = cuda(wk.sources())
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), U)
    yield wk, ctx, b
    ctx.close()
    torch.cuda.empty_cache()


def test_stencil_24x24x24x48(big):
    from paper_1010_2592_amd import msb
    wk, ctx, b = big
    fx = fixture()
    case = fx["cases"]["24x24x24x48 stencil"]
    fp = Fingerprint(fx, wk.dims, case["sample_seed"])
    log("24x24x24x48 stencil gamma5 D b")
    check("g5 D b", fp.errors(ctx.wilson_apply(b, msb.G5_LEFT), case["g5_dw_b"]), 1e-14)


@pytest.mark.parametrize("l,M", [(2, 2), (6, 1)])
def test_forced_parity_24x24x24x48(big, l, M):
    import torch
    from paper_1010_2592_amd import msb
    wk, ctx, b = big
    fx = fixture()
    case = fx["cases"][f"24x24x24x48 l={l} M={M}"]
    fp = Fingerprint(fx, wk.dims, case["sample_seed"])
    sig, w = msb.neuberger_pfe(wk.n_shift)
    force = np.full(len(sig), M)
    allow = (msb.OK, msb.NOT_CONVERGED)
    for name, pass_, fl, want in FORMS:
        flags = getattr(msb, fl) if fl else 0
        log(f"24x24x24x48 l={l}, {M} forced outer iterations: {name}")
        y, info, xs = ctx.mshift_bicgstabl(b, case["a_scale"], sig, w, l, wk.tol, M, pass_, flags=flags,
                                           want_shifts=want, force_iters=force, allow=allow)
        assert info.status == case["status"] and info.outer_iters == M
        check(f"{name} y", fp.errors(y, case["y"]), bound_of(case))
        if want:
            for s, ref in zip(case["shifts_kept"], case["x"]):
                check(f"{name} x_{s}", fp.errors(xs[0, s], ref), bound_of(case))
        del y, xs
        torch.cuda.empty_cache()


def test_forced_parity_headline_batch():
    import torch
    from paper_1010_2592_amd import msb
    wk = wl.WORKLOADS["16x16x16x32"]
    fx = fixture()
    log("16x16x16x32, 12 point sources, freeze iterations forced per (source, shift)")
    U = cuda(wk.links())
    b = cuda(wl.point_sources(wk.dims))
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), U)
    sig, w = msb.neuberger_pfe(wk.n_shift)
    F = force_16(12, len(sig))
    allow = (msb.OK, msb.NOT_CONVERGED)
    a = fx["cases"]["16x16x16x32 source 0"]["a_scale"]
    for name, pass_, fl, want in FORMS:
        flags = getattr(msb, fl) if fl else 0
        log(f"  {name}")
        y, info, xs = ctx.mshift_bicgstabl(b, a, sig, w, 4, wk.tol, 20, pass_, flags=flags, want_shifts=want,
                                           force_iters=F, allow=allow)
        assert np.all(info.shift_iters <= F)
        assert info.outer_iters == int(F.max())
        for r in (0, 6):
            case = fx["cases"][f"16x16x16x32 source {r}"]
            fp = Fingerprint(fx, wk.dims, case["sample_seed"])
            assert case["force"] == F[r].tolist() and case["outer"] == int(F[r].max())
            assert info.shift_iters[r].tolist() == case["shift_iters"]
            check(f"{name} source {r} y", fp.errors(y[r], case["y"]), bound_of(case))
            if want:
                for s, ref in zip(case["shifts_kept"], case["x"]):
                    check(f"{name} source {r} x_{s}", fp.errors(xs[r, s], ref), bound_of(case))
        del y, xs
        torch.cuda.empty_cache()
    ctx.close()
