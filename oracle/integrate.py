"""Explicit stepping of Eq. (3)-(4), the controller of Eq. (5) and the
polynomial extrapolation of the demagnetizing field of Eq. (6).

One iteration from (t0, M0) with step h:

  F_k = F(t0 + a_k h, M_k),  M_k = M0 + h sum_{l<k} b_kl F_l          (Eq. 4)
  M   = M0 + h sum_k c_k F_k,   M^ = M0 + h sum_k c^_k F_k            (Eq. 3)
  e   = ||M - M^|| / Ms, computed as ||h sum_k (c_k - c^_k) F_k|| / Ms

Readings of the paper taken here (the GPU library takes the same ones):

* e: the maximum over cells of the per-cell Euclidean norm.
* Eq. (5) exponent: the text reads "1/n+1" with n the method order.  Default
  ``exponent='min'`` uses 1/(q+1), q = min(n, n^) (the order of the local
  error estimate of an embedded pair); ``exponent='literal'`` uses
  1/(n+1) with n the propagated order.  Constants: h_min 1 fs, h_max 3 ps,
  c_min 0.01, c_max 2, e_max 1e-5, safety 0.8 (Sec. II).  A step with
  e > e_max is repeated from the same (t0, M0) with h' = max(h c, h_min);
  a step at h_min is accepted whatever e is.
* Eq. (6) sign: Eq. (2) defines H = -N M, so the self field of a cell is
  Hself(M) = -N00 M with N00 the (positive) self term.  The stored fields
  are G_i = H_i - Hself(M_i) and the extrapolated field is
  H(t) = sum_i G_i L_i(t) + Hself(M(t)): the self contribution is removed
  before extrapolation and added back at the current M, which is what the
  text around Eq. (6) describes.
* The one exact evaluation of Eq. (2) per iteration is at stage 1 (t0, M0),
  whose start time is t_i for the current iteration; the other nodes are the
  start times of the previous p accepted iterations.  Every other stage,
  including a stage at t0 + h of an FSAL tableau, is extrapolated.  The
  first p accepted iterations run with exact evaluation at every stage and
  store their stage-1 G (priming).  A rejected attempt reuses stage 1
  (it does not depend on h) and does not advance the history.
* Full evaluation (extrap=None): every stage is exact; an FSAL tableau
  reuses its last stage as the next stage 1 when ``renormalize`` is off.
* ``renormalize`` (off by default): rescale every cell to |M| = Ms after each
  accepted iteration (empty cells, M = 0, stay empty).

ABM2 (the 2nd-order Adams-Bashforth-Moulton predictor-corrector of Sec. II,
ref. [32]), in PECE form with the readings taken here:

* predictor, variable-step AB2 with r = h_n / h_{n-1}:
  M_p = M_n + h_n ((1 + r/2) F_n - (r/2) F_{n-1}); the first step after a
  start (no F_{n-1}) uses M_p = M_n + h F_n, i.e. Heun's method;
* E: F_p = F(t_n + h, M_p) -- with extrapolation this is the Eq. (6) field at
  t_n + h (nodes: the current and p previous iteration starts);
* corrector, trapezoidal (AM2): M_{n+1} = M_n + (h/2)(F_n + F_p);
* E: F_{n+1} = F(t_{n+1}, M_{n+1}) with exact Eq. (2): the one exact
  evaluation per iteration, whose stored field G and time are the next
  iteration's start node; it is evaluated after acceptance (and after
  renormalisation), so a rejected attempt costs one evaluation;
* error (Milne): the corrector's local error, -h^3/12 times the third time
  derivative of M, is estimated as r/(3(r+1)) |M_{n+1} - M_p| per cell, max
  over cells, / Ms; Heun's estimate |M_{n+1} - M_p| on the starting step;
  Eq. (5) exponent 1/3 (q = 2).

Pins (tests/test_oracle_integrate.py, test_oracle_extrap.py): convergence
order of every tableau on the closed-form damped precession; extrapolation
exact on polynomials of degree <= p for either sign reading; the single-cell
sign test; L_i at uniform spacing (sum |L_i| = 2^(p+1) - 1 at a = 1);
controller clamps and rejection; monotone energy decay under damping; |M|
conservation.
"""

import numpy as np

from . import demag as _demag
from . import fields as _fields
from .tableaux import TABLEAUX

H_MIN = 1e-15
H_MAX = 3e-12
C_MIN = 0.01
C_MAX = 2.0
E_MAX = 1e-5


def lagrange_weights(nodes, t):
    """L_i(t) = prod_{j != i} (t - t_j)/(t_i - t_j) of Eq. (6)."""
    nodes = [float(v) for v in nodes]
    w = []
    for i, ti in enumerate(nodes):
        li = 1.0
        for j, tj in enumerate(nodes):
            if j != i:
                li *= (t - tj) / (ti - tj)
        w.append(li)
    return np.array(w)


def stored_field(H, M, N00):
    """G = H - Hself(M) with Hself(M) = -N00 M (the stored fields of Eq. (6))."""
    return H + N00[:, None, None, None] * M


def extrapolated_field(nodes, Gs, t, Mt, N00):
    """Eq. (6): sum_i G_i L_i(t) + Hself(M(t))."""
    L = lagrange_weights(nodes, t)
    H = -N00[:, None, None, None] * Mt
    for Li, Gi in zip(L, Gs):
        H = H + Li * Gi
    return H


def controller_factor(e, e_max=E_MAX, q=4, c_min=C_MIN, c_max=C_MAX):
    """c of Eq. (5) with exponent 1/(q+1)."""
    if e <= 0.0:
        return c_max
    return min(max((0.8 * e_max / e) ** (1.0 / (q + 1)), c_min), c_max)


def controller_step(h, c, h_min=H_MIN, h_max=H_MAX):
    """h' of Eq. (5)."""
    return min(max(h * c, h_min), h_max)


def ab2_predict(M0, F0, Fprev, h, h_prev):
    """Variable-step AB2 predictor (Heun's Euler predictor without F_{n-1})."""
    if Fprev is None:
        return M0 + h * F0
    r = h / h_prev
    return M0 + h * ((1.0 + 0.5 * r) * F0 - (0.5 * r) * Fprev)


def am2_correct(M0, F0, Fp, h):
    """Trapezoidal (AM2) corrector."""
    return M0 + (0.5 * h) * (F0 + Fp)


def milne_factor(r):
    """Local error of the AM2 corrector over (corrector - AB2 predictor) for
    the step ratio r = h_n / h_{n-1}, on solutions with constant third
    derivative."""
    return r / (3.0 * (r + 1.0))


class Integrator:
    """State (t, M, h, history) and one-iteration stepping for a problem dict.

    extrap: None for full evaluation at every stage, an int p >= 0 for
    Eq. (6) of order p, or 'matched' for p = n (the propagated order).
    """

    def __init__(self, problem, M0, method="RK4", extrap=None, h=1e-13, adaptive=None,
                 h_min=H_MIN, h_max=H_MAX, c_min=C_MIN, c_max=C_MAX, e_max=E_MAX,
                 renormalize=False, exponent="min", Nfull=None, demag_fn=None, workers=None):
        self.pa = _fields.problem_arrays(problem)
        self.workers = workers  # threads of scipy.fft in Eq. (2) (None: one)
        self.multistep = method == "ABM2"
        if self.multistep:
            self.tab = None
            if extrap == "matched":
                extrap = 2
            self.adaptive = True if adaptive is None else bool(adaptive)
            self.q = 2
        else:
            self.tab = TABLEAUX[method]
            if extrap == "matched":
                extrap = self.tab.order
            self.adaptive = self.tab.adaptive if adaptive is None else bool(adaptive)
            if self.adaptive and not self.tab.adaptive:
                raise ValueError("method has no embedded estimate")
            if exponent == "min":
                self.q = min(self.tab.order, self.tab.order_hat) if self.tab.adaptive else self.tab.order
            else:
                self.q = self.tab.order
        self.p = extrap
        self.h_min, self.h_max, self.c_min, self.c_max, self.e_max = h_min, h_max, c_min, c_max, e_max
        self.renormalize = renormalize
        n = self.pa["n"]
        if Nfull is None:
            from . import newell
            Nfull = newell.tensor_full(n, self.pa["cell"])
        self.Nfull = Nfull
        c0 = (slice(None), n[2] - 1, n[1] - 1, n[0] - 1)
        self.N00 = np.array(Nfull[c0][:3])  # diagonal of N(0)
        self.Khat = _demag.kspace_kernel(Nfull, n)
        self.demag_fn = demag_fn
        self.t = 0.0
        self.M = np.array(M0, dtype=np.float64)
        self.h = float(h)
        self.hist = []        # previous accepted (t_i, G_i), oldest first, at most p
        self.fsal_F = None
        self.stats = dict(exact=0, extrap=0, accepted=0, rejected=0, forced=0)
        # ABM2 state: F_n and its stored field G_n at (t, M), F_{n-1} and h_{n-1}
        self.abm_F = self.abm_G = self.abm_Fprev = None
        self.abm_hprev = None
        if not self.multistep:
            self.a = [[float(v) for v in row] for row in self.tab.a]
            self.b = [float(v) for v in self.tab.b]
            self.c = [float(v) for v in self.tab.c]
            self.db = None if self.tab.bhat is None else [float(x - y) for x, y in zip(self.tab.b, self.tab.bhat)]

    # --- field evaluations -------------------------------------------------
    def demag(self, M):
        if self.demag_fn is not None:
            return self.demag_fn(M)
        return _demag.demag_fft(M, self.Nfull, self.Khat, workers=self.workers)

    def rhs(self, M, Hd):
        pa = self.pa
        H = _fields.effective_field(M, Hd, pa)
        return _fields.llg_rhs(M, H, pa["Ms"], pa["alpha"], pa["gamma"])

    def set_m(self, M):
        """New magnetization: the history is no longer valid and priming restarts."""
        self.M = np.array(M, dtype=np.float64)
        self.hist = []
        self.fsal_F = None
        self.abm_F = self.abm_G = self.abm_Fprev = None
        self.abm_hprev = None

    # --- one accepted iteration -------------------------------------------
    def step(self, h=None):
        if h is not None:
            self.h = float(h)
        if self.multistep:
            return self._step_abm()
        tab, p = self.tab, self.p
        M0, t0 = self.M, self.t
        use_extrap = p is not None and len(self.hist) == p
        if self.fsal_F is not None:
            F1 = self.fsal_F
            G0 = None
        else:
            Hd0 = self.demag(M0)
            self.stats["exact"] += 1
            F1 = self.rhs(M0, Hd0)
            G0 = stored_field(Hd0, M0, self.N00) if p is not None else None
        h = self.h
        if self.adaptive:
            h = min(max(h, self.h_min), self.h_max)
        rejected = 0
        forced = False
        while True:
            Fs = [F1]
            for k in range(1, tab.stages):
                Mk = M0.copy()
                for l in range(k):
                    if self.a[k][l] != 0.0:
                        Mk = Mk + (h * self.a[k][l]) * Fs[l]
                if use_extrap:
                    nodes = [ti - t0 for ti, _ in self.hist] + [0.0]
                    Gs = [g for _, g in self.hist] + [G0]
                    Hd = extrapolated_field(nodes, Gs, self.c[k] * h, Mk, self.N00)
                    self.stats["extrap"] += 1
                else:
                    Hd = self.demag(Mk)
                    self.stats["exact"] += 1
                Fs.append(self.rhs(Mk, Hd))
            Mnew = M0.copy()
            for k in range(tab.stages):
                if self.b[k] != 0.0:
                    Mnew = Mnew + (h * self.b[k]) * Fs[k]
            err = 0.0
            if self.db is not None:
                D = np.zeros_like(M0)
                for k in range(tab.stages):
                    if self.db[k] != 0.0:
                        D = D + (h * self.db[k]) * Fs[k]
                err = float(np.max(np.sqrt(np.sum(D * D, axis=0)))) / self.pa["Ms"]
            if self.adaptive:
                c = controller_factor(err, self.e_max, self.q, self.c_min, self.c_max)
                if err > self.e_max:
                    if h > self.h_min:
                        rejected += 1
                        h = controller_step(h, c, self.h_min, self.h_max)
                        continue
                    forced = True
                h_next = controller_step(h, c, self.h_min, self.h_max)
            else:
                h_next = h
            break
        # accept
        if p is not None:
            if G0 is None:  # cannot happen: FSAL reuse is off whenever p is set
                raise RuntimeError("missing stage-1 field")
            if p > 0:
                self.hist.append((t0, G0))
                self.hist = self.hist[-p:]
        if p is None and tab.fsal and not self.renormalize:
            self.fsal_F = Fs[-1]
        else:
            self.fsal_F = None
        if self.renormalize:
            Mnew = _fields.renormalized(Mnew, self.pa["Ms"])
        self.M = Mnew
        self.t = t0 + h
        self.h = h_next
        self.stats["accepted"] += 1
        self.stats["rejected"] += rejected
        self.stats["forced"] += int(forced)
        return dict(t=self.t, h_used=h, h_next=h_next, err=err, rejected=rejected, forced=forced)

    def _exact_start(self, M):
        Hd = self.demag(M)
        self.stats["exact"] += 1
        F = self.rhs(M, Hd)
        G = stored_field(Hd, M, self.N00) if self.p is not None else None
        return F, G

    def _step_abm(self):
        p = self.p
        M0, t0 = self.M, self.t
        if self.abm_F is None:
            self.abm_F, self.abm_G = self._exact_start(M0)
        F0, G0 = self.abm_F, self.abm_G
        use_extrap = p is not None and len(self.hist) == p
        h = self.h
        if self.adaptive:
            h = min(max(h, self.h_min), self.h_max)
        rejected = 0
        forced = False
        while True:
            Mp = ab2_predict(M0, F0, self.abm_Fprev, h, self.abm_hprev)
            if use_extrap:
                nodes = [ti - t0 for ti, _ in self.hist] + [0.0]
                Gs = [g for _, g in self.hist] + [G0]
                Hd = extrapolated_field(nodes, Gs, h, Mp, self.N00)
                self.stats["extrap"] += 1
            else:
                Hd = self.demag(Mp)
                self.stats["exact"] += 1
            Fp = self.rhs(Mp, Hd)
            Mc = am2_correct(M0, F0, Fp, h)
            D = Mc - Mp
            fac = 1.0 if self.abm_Fprev is None else milne_factor(h / self.abm_hprev)
            err = fac * float(np.max(np.sqrt(np.sum(D * D, axis=0)))) / self.pa["Ms"]
            if self.adaptive:
                c = controller_factor(err, self.e_max, self.q, self.c_min, self.c_max)
                if err > self.e_max:
                    if h > self.h_min:
                        rejected += 1
                        h = controller_step(h, c, self.h_min, self.h_max)
                        continue
                    forced = True
                h_next = controller_step(h, c, self.h_min, self.h_max)
            else:
                h_next = h
            break
        if p is not None and p > 0:
            self.hist.append((t0, G0))
            self.hist = self.hist[-p:]
        if self.renormalize:
            Mc = _fields.renormalized(Mc, self.pa["Ms"])
        self.abm_Fprev, self.abm_hprev = F0, h
        self.M = Mc
        self.t = t0 + h
        self.h = h_next
        self.abm_F, self.abm_G = self._exact_start(Mc)
        self.stats["accepted"] += 1
        self.stats["rejected"] += rejected
        self.stats["forced"] += int(forced)
        return dict(t=self.t, h_used=h, h_next=h_next, err=err, rejected=rejected, forced=forced)

    def run(self, t_end, sample_dt=None):
        """Step until t_end.  With sample_dt, record <M> at multiples of sample_dt;
        an adaptive step is shortened to land on the next sample time and the
        step after it resumes from the larger of the controller's proposal and
        the step size before shortening."""
        samples = []
        next_s = 0.0 if sample_dt else None
        if sample_dt:
            samples.append(self.mean_m())
            next_s = sample_dt
        tol = 1e-9 * self.h
        while self.t < t_end - tol:
            h_prop = self.h
            target = t_end if next_s is None else min(next_s, t_end)
            shortened = False
            if self.adaptive and self.t + self.h > target:
                self.h = target - self.t
                shortened = True
            info = self.step()
            if shortened:
                self.h = max(self.h, h_prop)
            if next_s is not None and self.t >= next_s - 1e-9 * info["h_used"]:
                samples.append(self.mean_m())
                next_s += sample_dt
        return np.array(samples)

    def mean_m(self):
        return self.M.reshape(3, -1).mean(axis=1)
