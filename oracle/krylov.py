"""BiCGstab(l), multi-shift BiCGstab(l) single-pass, and the double-pass form.

Test infrastructure only (see ``oracle/__init__.py``).

What is computed
----------------
f(A) b ~ sum_s w_s (A + sigma_s)^{-1} b  (Eq. (1.2)) from ONE Krylov space, by
the shift invariance K_k(A + sigma, b) = K_k(A, b) (Section 1).  The unshifted
("seed") iteration is BiCGstab(l) (Section 2; Sleijpen-Fokkema), run on the
seed matrix S = A + sigma_0 with sigma_0 = min_s sigma_s; every shifted system
(S + sigma'_s) x_s = b, sigma'_s = sigma_s - sigma_0 >= 0, reuses the seed's
vectors with collinear residuals (Frommer's shifted BiCGstab(l), cited in
Section 2).

Notation (polynomial view).  n = m*l + j counts BiCG steps (outer iteration
m, inner step j).  The seed's BiCG polynomials R_n, P_n obey
  P_n = R_n - beta_n P_{n-1},   R_{n+1} = R_n - alpha_n t P_n,
the MR ("minimal residual") polynomial of outer iteration m is
q_m(t) = 1 - sum_i gamma_i t^i, and r_0 = Q_m(S) R_n(S) b with
Q_m = prod_{k<m} q_k.  For a shift, zeta_n = R_n(-sigma'), pi_n = P_n(-sigma'),
psi = Q(-sigma'); its residual is r_0 / (zeta_n psi) (collinear), and
  alpha^s_n = alpha_n zeta_n / zeta_{n+1},  beta^s_n = beta_n (zeta_{n-1}/zeta_n)^2
follow from matching the three-term recurrences of R_n(t) and
R^s_n(t + sigma') = R_n(t) / zeta_n.  The shift's own MR polynomial is
q(t - sigma') / q(-sigma').

MR part: normal equations G gamma = c, G_ik = <r_i, r_k>, c_i = <r_i, r_0>
(i, k = 1..l), by Cholesky.  Its dot count, l(l+3)/2 per outer iteration, plus
two per BiCG step gives the paper's M l (0.5 l + 3.5) (Section 3 cost table).

Double-pass (Section 2, option 1 after Eq. (2.2); Section 5).  Pass 1 runs the
seed and the shifts' *scalar* recurrences only, recording the scalars.  The
single-pass program that forms sum_s w_s x_s is then a fixed linear program in
its sources -- b and the Mv outputs v_t -- so its coefficients c_b, c_t follow
from one backward (transposed) sweep over the recorded scalars.  Pass 2
regenerates the v_t from the recorded scalars (no dot products) and
accumulates y = c_b b + sum_t c_t v_t.  This reaches the same y as the
paper's closed-form coefficients of Section 5 in a different bookkeeping.

Inner product <a, b> = sum conj(a_i) b_i.  All arithmetic complex128/float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

# breakdown thresholds (relative)
BREAK_REL = 1e-14
CHOL_REL = 1e-14
ZETA_MIN = 1e-300
# a shift whose |zeta psi| would exceed ZETA_MAX has a residual estimate
# ||r_0|| / (|zeta psi| ||b||) below any tolerance (for any ||r_0|| within
# 1e20 of ||b||) and 1 / (zeta psi) would underflow: it stops there as
# converged, its solution complete to rounding
ZETA_MAX = 1e300
# outcome of a shift's scalar step
STEP_OK, STEP_BROKEN, STEP_DONE = 0, 1, 2
# a shift freezes once its recursive (collinear) residual estimate is at most
# FREEZE_FRAC * tol, so that the rounding drift between the recursive and the
# true residual (about 1e-15 relative in FP64) cannot lift the true residual
# of a frozen shift above tol (the paper's convergence test, Section 2, reads
# the residual of each shifted system; which estimate is not specified)
FREEZE_FRAC = 0.9

OK, NOT_CONVERGED, BREAKDOWN = 0, 4, 5


def dot(a, b) -> complex:
    return complex(np.vdot(a, b))


def norm(a) -> float:
    return float(np.sqrt(np.vdot(a, a).real))


def cholesky_solve(G: np.ndarray, c: np.ndarray):
    """Solve G g = c for Hermitian positive definite G by Cholesky.

    Returns (g, k): if a pivot falls below CHOL_REL * max diag at index k
    (0-based), only the leading k x k block is solved and k < len(c).
    """
    n = len(c)
    if n == 0:
        return np.zeros(0, dtype=np.complex128), 0
    dmax = max(G[i, i].real for i in range(n))
    L = np.zeros((n, n), dtype=np.complex128)
    k_ok = n
    for i in range(n):
        d = G[i, i].real - sum(abs(L[i, p]) ** 2 for p in range(i))
        if not (d > CHOL_REL * dmax):
            k_ok = i
            break
        L[i, i] = np.sqrt(d)
        for r in range(i + 1, n):
            L[r, i] = (G[r, i] - sum(L[r, p] * np.conj(L[i, p]) for p in range(i))) / L[i, i]
    n = k_ok
    # forward: L z = c ; backward: L^H g = z
    z = np.zeros(n, dtype=np.complex128)
    for i in range(n):
        z[i] = (c[i] - sum(L[i, p] * z[p] for p in range(i))) / L[i, i]
    g = np.zeros(n, dtype=np.complex128)
    for i in reversed(range(n)):
        g[i] = (z[i] - sum(np.conj(L[p, i]) * g[p] for p in range(i + 1, n))) / L[i, i].real
    return g, n


def mr_coefficients_normal(r):
    """gamma_1..gamma_l minimising ||r_0 - sum gamma_i r_i|| (normal eqs)."""
    l = len(r) - 1
    G = np.empty((l, l), dtype=np.complex128)
    c = np.empty(l, dtype=np.complex128)
    for i in range(1, l + 1):
        c[i - 1] = dot(r[i], r[0])
        for k in range(1, l + 1):
            G[i - 1, k - 1] = dot(r[i], r[k])
    return cholesky_solve(G, c)


# ---------------------------------------------------------------------------
# single system
# ---------------------------------------------------------------------------

def bicgstab_textbook(mv, b, tol, maxit):
    """van der Vorst's BiCGstab, x0 = 0, shadow = b.  Returns per-iteration x."""
    x = np.zeros_like(b)
    r = b.copy()
    rs = b.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    xs = []
    bn = norm(b)
    for _ in range(maxit):
        rho_new = dot(rs, r)
        beta = (rho_new / rho) * (alpha / omega)
        rho = rho_new
        p = r + beta * (p - omega * v)
        v = mv(p)
        alpha = rho / dot(rs, v)
        s = r - alpha * v
        t = mv(s)
        omega = dot(t, s) / dot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        xs.append(x.copy())
        if norm(r) <= tol * bn:
            break
    return xs


def bicg_textbook(A: np.ndarray, b, nsteps):
    """Plain BiCG (biconjugate gradient) on a dense matrix, shadow r~ = b.

    Returns the step lengths alpha_n and the direction coefficients beta_n in
    the convention p_n = r_n + beta_n p_{n-1}.
    """
    r = b.copy()
    rt = b.copy()
    p = r.copy()
    pt = rt.copy()
    alphas, betas = [], []
    rho = dot(rt, r)
    for _ in range(nsteps):
        Ap = A @ p
        alpha = rho / dot(pt, Ap)
        r = r - alpha * Ap
        rt = rt - np.conj(alpha) * (A.conj().T @ pt)
        rho_new = dot(rt, r)
        beta = rho_new / rho
        rho = rho_new
        p = r + beta * p
        pt = rt + np.conj(beta) * pt
        alphas.append(alpha)
        betas.append(beta)
    return np.array(alphas), np.array(betas)


@dataclass
class SeedInfo:
    outer: int = 0
    mv: int = 0
    alphas: List[complex] = field(default_factory=list)
    betas: List[complex] = field(default_factory=list)
    gammas: List[np.ndarray] = field(default_factory=list)
    xs: List[np.ndarray] = field(default_factory=list)
    status: int = OK


def bicgstabl(mv, b, l, tol, max_outer, mr="normal", keep_x=False):
    """BiCGstab(l) for S x = b with x0 = 0 and shadow residual r~ = b.

    ``mr`` selects the minimal-residual solve: "normal" (normal equations by
    Cholesky, as the library does) or "mgs" (Sleijpen-Fokkema's modified
    Gram-Schmidt form), a cross-check of the same minimisation.
    """
    info = SeedInfo()
    r = [b.copy()] + [np.zeros_like(b) for _ in range(l)]
    u = [np.zeros_like(b) for _ in range(l + 1)]
    x = np.zeros_like(b)
    rt = b.copy()
    bn = norm(b)
    rho0, alpha, omega = 1.0 + 0j, 0.0 + 0j, 1.0 + 0j
    for m in range(max_outer):
        rho0 = -omega * rho0
        for j in range(l):
            rho1 = dot(rt, r[j])
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = mv(u[j])
            info.mv += 1
            alpha = rho0 / dot(rt, u[j + 1])
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = mv(r[j])
            info.mv += 1
            x = x + alpha * u[0]
            info.alphas.append(alpha)
            info.betas.append(beta)
        if mr == "normal":
            g, _ = mr_coefficients_normal(r)
        else:
            g = _mr_mgs(r)
        info.gammas.append(g)
        for i in range(1, l + 1):
            x = x + g[i - 1] * r[i - 1]
        for i in range(1, l + 1):
            r[0] = r[0] - g[i - 1] * r[i]
            u[0] = u[0] - g[i - 1] * u[i]
        omega = g[l - 1]
        info.outer = m + 1
        if keep_x:
            info.xs.append(x.copy())
        if norm(r[0]) <= tol * bn:
            return x, info
    info.status = NOT_CONVERGED
    return x, info


def _mr_mgs(r):
    """MR coefficients by modified Gram-Schmidt (Sleijpen-Fokkema)."""
    l = len(r) - 1
    rr = [v.copy() for v in r]
    tau = np.zeros((l + 1, l + 1), dtype=np.complex128)
    sig = np.zeros(l + 1)
    gp = np.zeros(l + 1, dtype=np.complex128)
    for j in range(1, l + 1):
        for i in range(1, j):
            tau[i, j] = dot(rr[i], rr[j]) / sig[i]
            rr[j] = rr[j] - tau[i, j] * rr[i]
        sig[j] = dot(rr[j], rr[j]).real
        gp[j] = dot(rr[j], rr[0]) / sig[j]
    g = np.zeros(l + 1, dtype=np.complex128)
    g[l] = gp[l]
    for j in range(l - 1, 0, -1):
        g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, l + 1))
    return g[1:]


# ---------------------------------------------------------------------------
# multi-shift
# ---------------------------------------------------------------------------

@dataclass
class StepRec:
    """Recorded scalars of one BiCG step of the seed."""
    beta: complex
    alpha: Optional[complex]       # None: gamma breakdown after S u_j


@dataclass
class OuterRec:
    steps: List[StepRec]
    gammas: np.ndarray             # MR coefficients actually applied
    active: np.ndarray             # bool [N]: shifts updated in this iteration


@dataclass
class MShiftInfo:
    status: int = OK
    outer: int = 0
    mv: int = 0
    dots: int = 0
    steps: int = 0                        # BiCG steps (2 Mv each)
    shift_iters: np.ndarray = None        # M_s per shift (caller order)
    shift_resid: np.ndarray = None        # final collinear residual estimate
    tape: List[OuterRec] = field(default_factory=list)
    coeff_b: complex = 0j
    coeff_v: np.ndarray = None            # c_t per Mv output (double-pass)
    shift_breakdown: np.ndarray = None


class _ShiftScalars:
    """Per-shift scalar recurrences of the shifted BiCGstab(l)."""

    def __init__(self, sp):
        n = len(sp)
        self.sp = np.asarray(sp, dtype=np.float64)      # sigma'
        self.zeta = np.ones(n, dtype=np.complex128)      # zeta_n
        self.zeta_prev = np.ones(n, dtype=np.complex128)  # zeta_{n-1}
        self.pi_prev = np.zeros(n, dtype=np.complex128)  # pi_{n-1}
        self.psi = np.ones(n, dtype=np.complex128)       # prod_k q_k(-sigma')

    def bicg_step(self, s, alpha, beta):
        """Advance shift s over seed step (alpha_n, beta_n).

        Returns (STEP_OK, (alpha_s, beta_s, kappa_n, kappa_{n+1})), or
        (STEP_BROKEN, None) when zeta_{n+1} = zeta_n + alpha sigma' pi_n is not
        finite or cancels to rounding (the shifted BiCG recurrence has no
        next iterate), or (STEP_DONE, None) when |zeta_{n+1} psi| exceeds
        ZETA_MAX (converged; see ZETA_MAX).
        """
        z, zp, pp, ps = self.zeta[s], self.zeta_prev[s], self.pi_prev[s], self.psi[s]
        pi_n = z - beta * pp
        step = alpha * self.sp[s] * pi_n
        z_next = z + step
        with np.errstate(over="ignore", invalid="ignore"):
            big = not abs(z_next) * abs(ps) <= ZETA_MAX
            if not np.isfinite(z_next) or abs(z_next) < ZETA_MIN or \
                    abs(z_next) <= BREAK_REL * (abs(z) + abs(step)):
                return STEP_BROKEN, None
        if big:
            return STEP_DONE, None
        alpha_s = alpha * z / z_next
        beta_s = beta * (zp / z) ** 2
        kap = 1.0 / (z * ps)
        kap_next = 1.0 / (z_next * ps)
        self.zeta_prev[s], self.zeta[s], self.pi_prev[s] = z, z_next, pi_n
        return STEP_OK, (alpha_s, beta_s, kap, kap_next)

    def mr_step(self, s, gammas):
        """Shift s's MR data: (STEP_OK, (q^s, c^s_k for k = 0..l'-1, kappa_n)),
        then psi *= q; or (STEP_BROKEN, None) when q^s = 1 - sum gamma_i
        (-sigma')^i is not finite or cancels to rounding, or (STEP_DONE, None)
        when |zeta psi q| exceeds ZETA_MAX."""
        sp = self.sp[s]
        lm = len(gammas)
        terms = [gammas[i - 1] * (-sp) ** i for i in range(1, lm + 1)]
        q = 1.0 - sum(terms)
        with np.errstate(over="ignore", invalid="ignore"):
            big = not abs(self.zeta[s]) * abs(self.psi[s]) * abs(q) <= ZETA_MAX
            if not np.isfinite(q) or abs(q) < ZETA_MIN or \
                    abs(q) <= BREAK_REL * (1.0 + sum(abs(t) for t in terms)):
                return STEP_BROKEN, None
        if big:
            return STEP_DONE, None
        c = np.array([sum(gammas[i - 1] * (-sp) ** (i - 1 - k) for i in range(k + 1, lm + 1)) / q
                      for k in range(lm)], dtype=np.complex128)
        kap = 1.0 / (self.zeta[s] * self.psi[s])
        self.psi[s] = self.psi[s] * q
        return STEP_OK, (q, c, kap)

    def resid_scale(self, s):
        return abs(self.zeta[s] * self.psi[s])


def mshift_bicgstabl(a_mv: Callable, b: np.ndarray, sigmas, weights, l: int,
                     tol: float, max_outer: int, pass_: int = 1,
                     force_iters=None, monitor=None, keep_shifts=False, shadow=None, trace=None):
    """f(A) b ~ sum_s w_s (A + sigma_s)^{-1} b by multi-shift BiCGstab(l).

    a_mv      callable v -> A v
    sigmas    shifts sigma_s (caller order, real >= 0 in the PFE use)
    weights   w_s
    pass_     1: single-pass (keeps N_s (l+1) shift vectors, Section 2);
              2: double-pass (no shift vectors; 4 M l Mv, Section 3 table)
    force_iters  optional per-shift M_s (test hook: freeze shift s after
              exactly that many outer iterations instead of testing res_s)
    monitor   optional callback(m, r0, X, scal, active) after each outer
              iteration (single-pass only), for the collinearity checks.
    shadow    optional shadow residual r~ (default r~ = b).  BiCGstab(l)
              admits any r~ with <r~, r_0> != 0; a point source with
              r~ = b meets a structural breakdown on D_w, whose hopping
              term changes the site parity.
    trace     optional list; for each outer iteration one dict is appended
              with the MR step's inputs (copies of r_0..r_L before the
              update), the coefficients applied and the number of completed
              BiCG steps -- instrumentation for tests, no effect on the
              iteration.

    Returns (y, info) for pass 2 and (y, info, xs) for pass 1 (xs the
    per-shift solutions in caller order).
    """
    sigmas = np.asarray(sigmas, dtype=np.float64)
    weights = np.asarray(weights, dtype=np.float64)
    N = len(sigmas)
    sig0 = float(sigmas.min())
    sp = sigmas - sig0

    def S(v):
        return a_mv(v) + sig0 * v

    info = MShiftInfo()
    info.shift_iters = np.zeros(N, dtype=np.int64)
    info.shift_resid = np.full(N, np.inf)
    info.shift_breakdown = np.zeros(N, dtype=bool)
    vectors = pass_ == 1

    r = [b.astype(np.complex128).copy()] + [np.zeros_like(b, dtype=np.complex128) for _ in range(l)]
    u = [np.zeros_like(r[0]) for _ in range(l + 1)]
    rt = r[0].copy() if shadow is None else np.asarray(shadow, dtype=np.complex128).copy()
    bn = norm(b)
    if vectors:
        X = [np.zeros_like(r[0]) for _ in range(N)]
        W = [[np.zeros_like(r[0]) for _ in range(l + 1)] for _ in range(N)]
    scal = _ShiftScalars(sp)
    active = np.ones(N, dtype=bool)
    rho0, alpha, omega = 1.0 + 0j, 0.0 + 0j, 1.0 + 0j
    seed_broken = False
    # tape of per-step per-shift scalars for the sweep (double-pass)
    shift_tape = []

    if bn == 0.0:
        info.status = OK
        active[:] = False

    for m in range(max_outer):
        if not active.any():
            break
        rho0 = -omega * rho0
        rec = OuterRec(steps=[], gammas=np.zeros(0, dtype=np.complex128), active=active.copy())
        mtape = {"steps": [], "mr": None}
        l_eff = l
        exhausted = False
        for j in range(l):
            if j >= 1 and force_iters is None:
                # Krylov space exhausted: every active shift already meets
                # its tolerance after the previous step's r-update
                lim = FREEZE_FRAC * tol * bn * min(scal.resid_scale(s) for s in np.nonzero(active)[0])
                if rn0 <= lim:
                    exhausted, l_eff = True, j
                    break
            rho1 = dot(rt, r[j])
            info.dots += 1
            if rho1 == 0 or not np.isfinite(rho1) or \
                    abs(rho1) <= BREAK_REL * norm(rt) * norm(r[j]):
                l_eff, seed_broken = j, True
                break
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = S(u[j])
            info.mv += 1
            gam = dot(rt, u[j + 1])
            info.dots += 1
            if gam == 0 or not np.isfinite(gam) or \
                    abs(gam) <= BREAK_REL * norm(rt) * norm(u[j + 1]):
                rec.steps.append(StepRec(beta, None))
                l_eff, seed_broken = j, True
                break
            alpha = rho0 / gam
            rec.steps.append(StepRec(beta, alpha))
            # shifted systems (uses r_i before this step's update)
            stape = {}
            for s in np.nonzero(active)[0]:
                kind, res = scal.bicg_step(s, alpha, beta)
                if kind != STEP_OK:
                    # the shift stops here (converged, or broken)
                    active[s] = False
                    info.shift_breakdown[s] = kind == STEP_BROKEN
                    info.shift_iters[s] = m
                    continue
                alpha_s, beta_s, kap, kap_next = res
                stape[s] = res
                if vectors:
                    Ws = W[s]
                    for i in range(j + 1):
                        Ws[i] = kap * r[i] - beta_s * Ws[i]
                    X[s] = X[s] + alpha_s * Ws[0]
                    r_new = r[j] - alpha * u[j + 1]
                    Ws[j + 1] = (kap * r[j] - kap_next * r_new) / alpha_s - sp[s] * Ws[j]
            mtape["steps"].append(stape)
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            rn0 = norm(r[0])            # fused into the r-update on the GPU
            r[j + 1] = S(r[j])
            info.mv += 1
            info.steps += 1

        # MR part over r_0 .. r_{l_eff}
        if exhausted:
            g, l_mr = np.zeros(0, dtype=np.complex128), l
        elif l_eff >= 1:
            g, l_mr = mr_coefficients_normal(r[: l_eff + 1])
            info.dots += l_eff * (l_eff + 3) // 2
        else:
            g, l_mr = np.zeros(0, dtype=np.complex128), 0
        if l_mr < l:
            seed_broken = True
        if trace is not None:
            trace.append({"r": [v.copy() for v in r[: l_eff + 1]], "gammas": g.copy(), "l_eff": l_eff,
                          "exhausted": exhausted, "steps": len(rec.steps)})
        rec.gammas = g.copy()
        smr = {}
        for s in np.nonzero(active)[0]:
            kind, res = scal.mr_step(s, g)
            if kind != STEP_OK:
                active[s] = False
                info.shift_breakdown[s] = kind == STEP_BROKEN
                info.shift_iters[s] = m
                continue
            q, c, kap = res
            smr[s] = res
            if vectors:
                for k in range(len(g)):
                    X[s] = X[s] + kap * c[k] * r[k]
                Ws = W[s]
                w0 = Ws[0]
                for i in range(1, len(g) + 1):
                    w0 = w0 - g[i - 1] * Ws[i]
                Ws[0] = w0 / q
        mtape["mr"] = smr
        for i in range(1, len(g) + 1):
            r[0] = r[0] - g[i - 1] * r[i]
            u[0] = u[0] - g[i - 1] * u[i]
        if len(g) == l:
            omega = g[l - 1]
        info.tape.append(rec)
        shift_tape.append(mtape)
        info.outer = m + 1

        # convergence test and freezing at the end of the outer iteration
        rn = norm(r[0])
        for s in np.nonzero(active)[0]:
            res_s = rn / (scal.resid_scale(s) * bn)
            info.shift_resid[s] = res_s
            done = (m + 1 >= force_iters[s]) if force_iters is not None else (res_s <= FREEZE_FRAC * tol)
            done = done or exhausted
            if done:
                active[s] = False
                info.shift_iters[s] = m + 1
        if monitor is not None and vectors:
            monitor(m, r[0], X, scal, rec.active)
        if seed_broken or exhausted:
            break

    if active.any():
        for s in np.nonzero(active)[0]:
            info.shift_iters[s] = info.outer
        info.status = BREAKDOWN if seed_broken else NOT_CONVERGED
    elif info.shift_breakdown.any():
        info.status = BREAKDOWN
    else:
        info.status = OK

    if vectors:
        y = np.zeros_like(r[0])
        for s in range(N):
            y = y + weights[s] * X[s]
        if keep_shifts:
            return y, info, X
        return y, info, X

    # ---- double-pass: transposed sweep, then the replay -------------------
    cb, cv = _sweep(info.tape, shift_tape, sp, weights, l)
    info.coeff_b, info.coeff_v = cb, cv
    y = _replay(S, b, info.tape, cb, cv, l, info)
    return y, info


def _sweep(tape, shift_tape, sp, weights, l):
    """Coefficients of sum_s w_s x_s on the sources b and v_t.

    Walks the single-pass program backwards.  Each program variable (seed
    r_i, u_i; shift u^s_i; x^s) carries the coefficient lam with which its
    current value enters the output.  An assignment v <- a v + b u gives
    lam(u) += b lam(v), lam(v) <- a lam(v); an Mv output v_t ends its
    variable's history: c_t = lam(v), lam(v) = 0.  lam(x^s) = w_s.
    """
    N = len(sp)
    lamR = np.zeros(l + 1, dtype=np.complex128)
    lamU = np.zeros(l + 1, dtype=np.complex128)
    lamW = np.zeros((N, l + 1), dtype=np.complex128)
    # enumerate Mv outputs in program order
    nmv = 0
    for rec in tape:
        for st in rec.steps:
            nmv += 1 if st.alpha is None else 2
    cv = np.zeros(nmv, dtype=np.complex128)
    t = nmv
    for rec, mt in zip(reversed(tape), reversed(shift_tape)):
        g = rec.gammas
        lm = len(g)
        # MR, reversed: u_0 update, r_0 update, then the shifts
        for i in range(1, lm + 1):
            lamU[i] += -g[i - 1] * lamU[0]
        for i in range(1, lm + 1):
            lamR[i] += -g[i - 1] * lamR[0]
        for s, (q, c, kap) in mt["mr"].items():
            for i in range(1, lm + 1):
                lamW[s, i] += -g[i - 1] * lamW[s, 0] / q
            lamW[s, 0] = lamW[s, 0] / q
            for k in range(lm):
                lamR[k] += kap * c[k] * weights[s]
        # BiCG steps, reversed
        nsteps = len(rec.steps)
        for j in reversed(range(nsteps)):
            st = rec.steps[j]
            if st.alpha is not None:
                # r_{j+1} <- S r_j
                t -= 1
                cv[t] = lamR[j + 1]
                lamR[j + 1] = 0
                # r_i <- r_i - alpha u_{i+1}
                for i in range(j + 1):
                    lamU[i + 1] += -st.alpha * lamR[i]
                # shifts
                for s, (alpha_s, beta_s, kap, kap_next) in mt["steps"][j].items():
                    a1 = (kap - kap_next) / alpha_s
                    a2 = kap_next * st.alpha / alpha_s
                    lamR[j] += a1 * lamW[s, j + 1]
                    lamU[j + 1] += a2 * lamW[s, j + 1]
                    lamW[s, j] += -sp[s] * lamW[s, j + 1]
                    lamW[s, j + 1] = 0
                    lamW[s, 0] += alpha_s * weights[s]
                    for i in range(j + 1):
                        lamR[i] += kap * lamW[s, i]
                        lamW[s, i] = -beta_s * lamW[s, i]
            # u_{j+1} <- S u_j
            t -= 1
            cv[t] = lamU[j + 1]
            lamU[j + 1] = 0
            # u_i <- r_i - beta u_i
            for i in range(j + 1):
                lamR[i] += lamU[i]
                lamU[i] = -st.beta * lamU[i]
    assert t == 0
    return lamR[0], cv


def _replay(S, b, tape, cb, cv, l, info):
    """Pass 2: regenerate the seed vectors from the recorded scalars."""
    r = [b.astype(np.complex128).copy()] + [np.zeros_like(b, dtype=np.complex128) for _ in range(l)]
    u = [np.zeros_like(r[0]) for _ in range(l + 1)]
    y = cb * r[0]
    t = 0
    for rec in tape:
        for j, st in enumerate(rec.steps):
            for i in range(j + 1):
                u[i] = r[i] - st.beta * u[i]
            u[j + 1] = S(u[j])
            info.mv += 1
            y = y + cv[t] * u[j + 1]
            t += 1
            if st.alpha is None:
                break
            for i in range(j + 1):
                r[i] = r[i] - st.alpha * u[i + 1]
            r[j + 1] = S(r[j])
            info.mv += 1
            y = y + cv[t] * r[j + 1]
            t += 1
        g = rec.gammas
        for i in range(1, len(g) + 1):
            r[0] = r[0] - g[i - 1] * r[i]
            u[0] = u[0] - g[i - 1] * u[i]
    return y
