"""Offline stage of Polar Express in FP64 (test infrastructure, see package doc).

Follows:
* Theorem 1 (Section 3.1, eqs. greedy / optimal / newbounds): the optimal
  composition is built greedily; each p_t is the odd-quintic minimax
  approximation of the constant 1 on [l_t, u_t]; then l_{t+1} = p_t(l_t) and
  u_{t+1} = 2 - l_{t+1}.
* Appendix E, eq. (linearsystem) and Algorithm 3: for a trial set
  {l, x1, x2, u} solve the 4x4 system p(l)=1-E, p(x1)=1+E, p(x2)=1-E, p(u)=1+E,
  then move x1, x2 to the interior critical points of p (roots of
  5c x^4 + 3b x^2 + a, quadratic in y = x^2); stop when |E| stops changing.
  When l/u is within 1 - 5e-6 of 1 the answer is the Newton-Schulz quintic
  scaled to u (the degenerate branch of Algorithm 3).
* Appendix E, eq. (deg3_solution): closed form for degree 3.
* Section 3.4 / Appendix F: safety factor p(x/1.01) and cushioning of the
  lower end of the design interval.  Appendix F states the cushion as a ratio
  rule ("select the update as though l_t = u_t/10") and says its code uses a
  different factor; the printed coefficient table is reproduced by the ratio
  rule applied to the image: the design interval [r u_t, u_t] is widened until
  its minimax quintic maps it onto an interval of ratio 1/10, i.e. r is the
  root of E(r) = 9/11 (``ratio_cushion``), followed by a rescaling that
  re-centres p(l_t) and p(u_t) about 1.

Readings where the paper is inconsistent (recorded in the design doc):
* the degenerate branch uses Algorithm 3's threshold l/u >= 1 - eps^(1/3)
  (eps = 1.11e-16); the exchange stops when |E| changes by at most 16 eps
  (the rounding level of the 4x4 solve);
* when a step is degenerate we emit the exact Newton-Schulz quintic
  (15/8, -10/8, 3/8), which is what the printed coefficient table holds;
* l_{t+1} is computed from the polynomial *before* the safety factor is
  applied; the safety factor is applied to every non-degenerate step
  (the printed table exempts only its Newton-Schulz entry);
* Algorithm 3 prints (x_2^{(1)})^5 in the system matrix; we read x_2^{(k)}.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EPS_DOUBLE = 1.11e-16                      # Algorithm 3's machine epsilon
SAFETY = 1.01
DEGENERATE_RATIO = 1.0 - EPS_DOUBLE ** (1.0 / 3.0)
NS5 = (15.0 / 8.0, -10.0 / 8.0, 3.0 / 8.0)


def eval_odd_quintic(abc, x):
    """p(x) = a x + b x^3 + c x^5 (Section 3.5, Horner form)."""
    a, b, c = abc
    x = np.asarray(x, dtype=np.float64)
    y = x * x
    return x * (a + y * (b + c * y))


@dataclass
class RemezResult:
    a: float
    b: float
    c: float
    E: float
    iters: int
    points: tuple = field(default_factory=tuple)
    degenerate: bool = False


def _solve_refined(M, r):
    """Solve the 4x4 system of eq. (linearsystem) with one step of iterative
    refinement, the residual taken in extended precision: as l/u -> 1 the
    system's condition number grows (Appendix E notes it; ~2e6 on the seventh
    step of the l = 1e-3 schedule), and a plain float64 solve then loses six
    digits of the coefficients."""
    z = np.linalg.solve(M, r)
    res = (np.asarray(r, dtype=np.longdouble)
           - np.asarray(M, dtype=np.longdouble) @ np.asarray(z, dtype=np.longdouble))
    return z + np.linalg.solve(M, res.astype(np.float64))


# Algorithm 3 repeats the exchange until |E| stops changing; in float64 the
# change bottoms out at the rounding level of the 4x4 solve (a few ulps of E,
# and a cycle between two values two ulps apart never meets an eps test), so
# the exchange stops once |E| moves by at most 16 eps.
REMEZ_TOL = 16 * EPS_DOUBLE


def remez_quintic(lo: float, hi: float, tol: float = REMEZ_TOL, max_iter: int = 100) -> RemezResult:
    """Minimax odd quintic approximation of 1 on [lo, hi] (Appendix E, Alg. 3).

    Returns the coefficients, the levelled error E of the last exchange and the
    number of exchanges.  ``points`` holds the final trial set (lo, x1, x2, hi).
    """
    if not (lo > 0.0 and hi > 0.0):
        raise ValueError("need 0 < lo, 0 < hi")
    # converged bounds (l_t ~ u_t, possibly crossed by one rounding) are degenerate
    if lo / hi >= DEGENERATE_RATIO:
        a, b, c = NS5[0] / hi, NS5[1] / hi ** 3, NS5[2] / hi ** 5
        return RemezResult(a, b, c, float("nan"), 0, (lo, hi), True)
    # initial interior trial points: they become exact as lo -> hi
    x1 = 0.75 * lo + 0.25 * hi
    x2 = 0.25 * lo + 0.75 * hi
    prev = math.inf
    it = 0
    while True:
        it += 1
        pts = np.array([lo, x1, x2, hi])
        # columns: x, x^3, x^5, alternating sign for the levelled error
        M = np.stack([pts, pts ** 3, pts ** 5, np.array([1.0, -1.0, 1.0, -1.0])], axis=1)
        a, b, c, E = _solve_refined(M, np.ones(4))
        # critical points of p: 5c y^2 + 3b y + a = 0, y = x^2
        disc = math.sqrt(9.0 * b * b - 20.0 * a * c)
        y_small = (-3.0 * b - disc) / (10.0 * c)
        y_large = (-3.0 * b + disc) / (10.0 * c)
        x1, x2 = math.sqrt(y_small), math.sqrt(y_large)
        if abs(abs(E) - abs(prev)) <= tol or it >= max_iter:
            break
        prev = E
    return RemezResult(float(a), float(b), float(c), float(E), it, (lo, x1, x2, hi), False)


def ratio_cushion(ratio: float = 0.1) -> float:
    """The cushion r of Appendix F's ratio rule applied to the image: the
    minimax quintic for 1 on [r, 1] has levelled error E with
    (1 - E) / (1 + E) = ratio, i.e. E = (1 - ratio) / (1 + ratio) (9/11 for
    the ratio 1/10).  E(r) decreases as r grows (the interval shrinks), so the
    root is bracketed and found by bisection to the spacing of doubles; the
    minimax error on [r u, u] does not depend on u."""
    target = (1.0 - ratio) / (1.0 + ratio)
    a, b = 1e-6, 0.5
    assert abs(remez_quintic(a, 1.0).E) > target > abs(remez_quintic(b, 1.0).E)
    while True:
        mid = 0.5 * (a + b)
        if mid <= a or mid >= b:
            break
        if abs(remez_quintic(mid, 1.0).E) > target:
            a = mid
        else:
            b = mid
    return 0.5 * (a + b)


# cushion factor of the default schedule (Appendix F's ratio rule, see above)
CUSHION = ratio_cushion(0.1)


def cubic_closed_form(lo: float, hi: float):
    """Degree-3 minimax approximation of 1 on [lo, hi], eq. (deg3_solution).

    p(x) = beta * p_NS(alpha x), p_NS(x) = 3/2 x - 1/2 x^3,
    alpha = sqrt(3 / (hi^2 + lo hi + lo^2)), beta = 4 / (2 + lo hi (lo + hi) alpha^3).
    Returns (a, b) of p(x) = a x + b x^3 and the error E = beta - 1.
    """
    alpha = math.sqrt(3.0 / (hi * hi + lo * hi + lo * lo))
    beta = 4.0 / (2.0 + lo * hi * (lo + hi) * alpha ** 3)
    return beta * 1.5 * alpha, -beta * 0.5 * alpha ** 3, beta - 1.0


@dataclass
class Schedule:
    abc: np.ndarray          # (T, 3) coefficients actually applied online
    abc_unsafe: np.ndarray   # (T, 3) before the safety factor
    ell: np.ndarray          # (T+1,) lower bounds l_1..l_{T+1}
    u: np.ndarray            # (T+1,) upper bounds u_1..u_{T+1}
    degenerate: np.ndarray   # (T,) bool, step emitted the exact NS5 quintic
    remez_iters: np.ndarray  # (T,) exchanges used

    @property
    def err_bound(self) -> float:
        """1 - l_{T+1}: the worst-case error of the composite (eq. optimal)."""
        return float(1.0 - self.ell[-1])


def greedy_schedule(ell: float, T: int, cushion: float = CUSHION, recentre: bool = True,
                    safety: float = SAFETY, safety_on_last: bool = True,
                    tenth_rule: bool = False) -> Schedule:
    """The offline stage of Algorithm 1 for d = 5 (Theorem 1 + Appendix F).

    ``cushion`` = c designs p_t on [max(l_t, c u_t), u_t]; 0 gives the pure
    greedy composition of Theorem 1.  ``tenth_rule`` designs on
    [max(l_t, u_t/10), u_t] as Algorithm 1 states, without re-centring.
    ``recentre`` rescales p_t so that p(l_t) + p(u_t) = 2.  ``safety`` replaces
    p_t(x) by p_t(x/safety) for non-degenerate steps (all of them, or all but
    the last when ``safety_on_last`` is False).
    """
    if not (0.0 < ell < 1.0) or T < 1:
        raise ValueError("need 0 < ell < 1 and T >= 1")
    l_t, u_t = float(ell), 1.0
    ells, us = [l_t], [u_t]
    unsafe, degen, iters = [], [], []
    for _ in range(T):
        if tenth_rule:
            lo = max(l_t, u_t / 10.0)
        else:
            lo = max(l_t, cushion * u_t)
        r = remez_quintic(lo, u_t)
        if r.degenerate:
            abc = NS5
        else:
            abc = (r.a, r.b, r.c)
            if recentre and not tenth_rule:
                k = 2.0 / (float(eval_odd_quintic(abc, l_t)) + float(eval_odd_quintic(abc, u_t)))
                abc = (abc[0] * k, abc[1] * k, abc[2] * k)
        unsafe.append(abc)
        degen.append(r.degenerate)
        iters.append(r.iters)
        l_t = float(eval_odd_quintic(abc, l_t))
        u_t = 2.0 - l_t
        ells.append(l_t)
        us.append(u_t)
    safe = []
    for t, (abc, dg) in enumerate(zip(unsafe, degen)):
        apply = (not dg) and (safety != 1.0) and (safety_on_last or t < T - 1)
        if apply:
            abc = (abc[0] / safety, abc[1] / safety ** 3, abc[2] / safety ** 5)
        safe.append(abc)
    return Schedule(np.array(safe), np.array(unsafe), np.array(ells), np.array(us),
                    np.array(degen), np.array(iters))


def greedy_schedule_cubic(ell: float, T: int, safety: float = SAFETY,
                          safety_on_last: bool = True) -> Schedule:
    """The greedy composition of Theorem 1 for degree 3: each p_t is the
    closed-form minimax cubic of eq. (deg3_solution) on [l_t, u_t]; its error
    equioscillates at l_t, 1/alpha and u_t, so the image is [1 - E, 1 + E]
    and l_{t+1} = 1 - E, u_{t+1} = 1 + E = 2 - l_{t+1} (eq. newbounds).  No
    cushion (every interval's cubic has p(x)/x decreasing on [0, u_t], so no
    value is pulled below the next lower bound); the safety factor of
    Appendix F as for degree 5.  Coefficients as (a, b, 0) triples."""
    if not (0.0 < ell < 1.0) or T < 1:
        raise ValueError("need 0 < ell < 1 and T >= 1")
    l_t, u_t = float(ell), 1.0
    ells, us, unsafe = [l_t], [u_t], []
    for _ in range(T):
        a, b, E = cubic_closed_form(l_t, u_t)
        unsafe.append((a, b, 0.0))
        l_t = float(eval_odd_quintic((a, b, 0.0), l_t))
        u_t = 2.0 - l_t
        ells.append(l_t)
        us.append(u_t)
    safe = []
    for t, abc in enumerate(unsafe):
        if safety != 1.0 and (safety_on_last or t < T - 1):
            abc = (abc[0] / safety, abc[1] / safety ** 3, 0.0)
        safe.append(abc)
    z = np.zeros(T, dtype=bool)
    return Schedule(np.array(safe), np.array(unsafe), np.array(ells), np.array(us), z,
                    np.zeros(T, dtype=int))


def composite(abc_list, x):
    """phi_T(x) = p_T(...p_1(x)) on scalars/arrays (eq. composition)."""
    y = np.asarray(x, dtype=np.float64)
    for abc in abc_list:
        y = eval_odd_quintic(abc, y)
    return y


def extend_schedule(abc, steps: int) -> np.ndarray:
    """Steps past the end of a table repeat its last triple (Appendix A.1)."""
    abc = np.asarray(abc, dtype=np.float64).reshape(-1, 3)
    if steps <= abc.shape[0]:
        return abc[:steps].copy()
    extra = np.repeat(abc[-1:], steps - abc.shape[0], axis=0)
    return np.concatenate([abc, extra], axis=0)


def remez_quintic_mp(lo, hi, dps: int = 50):
    """The same exchange as ``remez_quintic`` carried out in ``dps``-digit
    arithmetic (mpmath).  Used to bound the float64 rounding error of the
    4x4 solve, which grows as lo/hi -> 1 (Appendix E notes the ill-conditioning)."""
    import mpmath as mp
    with mp.workdps(dps):
        lo, hi = mp.mpf(lo), mp.mpf(hi)
        x1 = (3 * lo + hi) / 4
        x2 = (lo + 3 * hi) / 4
        prev = mp.inf
        tol = mp.mpf(10) ** (-(dps - 10))
        for _ in range(200):
            pts = [lo, x1, x2, hi]
            M = mp.matrix([[p, p ** 3, p ** 5, sg] for p, sg in zip(pts, [1, -1, 1, -1])])
            a, b, c, E = mp.lu_solve(M, mp.matrix([1, 1, 1, 1]))
            disc = mp.sqrt(9 * b * b - 20 * a * c)
            x1 = mp.sqrt((-3 * b - disc) / (10 * c))
            x2 = mp.sqrt((-3 * b + disc) / (10 * c))
            if abs(abs(E) - abs(prev)) < tol:
                break
            prev = E
        return a, b, c, E
