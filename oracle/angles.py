"""Plain reference of the angle-finding outer loop (Sec. 2.3; the find_angles calls of Sec. 3).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: shares no code with the library.

The paper names the methods (BFGS to the nearest local optimum, basinhopping, seeding round p
with the round p-1 angles, random restarts from uniform angles in [0, 2 pi)) and leaves their
details open; this file writes out the textbook versions, one start or chain at a time, in
numpy FP64, on the oracle's <C> and adjoint gradient:

* BFGS in inverse-Hessian form (Nocedal and Wright, Numerical Optimization, Alg. 6.1 with the
  update of their Eq. 6.17), H_0 = I rescaled to (s.y / y.y) I before the first update (their
  Eq. 6.20), an update skipped when s.y <= 1e-10 |s| |y|; backtracking line search by halving
  (their Alg. 3.1), at most 20 halvings, accepting a step on sufficient decrease (c1 = 1e-4)
  or on the approximate Wolfe conditions of Hager and Zhang (SIAM J. Optim. 16, 170 (2005);
  sigma = 0.9, delta = 0.1, eps = 1e-6); first trial step min(1, 1 / max|d|) along the
  search direction d (no angle moves more than one radian in a trial); converged when
  max|g| <= gtol max(1, |f|).
* Basinhopping (Wales and Doye, J. Phys. Chem. A 101, 5111 (1997)): local minimisation,
  uniform perturbation in [-step, step] per angle, local minimisation, Metropolis acceptance
  with probability exp(-(f_new - f_cur) / T).
* Round seeding: the previous optimum padded with a zero layer, and the INTERP resampling of
  Zhou, Wang, Choi, Pichler and Lukin, Phys. Rev. X 10, 021067 (2020).
* Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) as a counter-based
  generator, so that both implementations draw the same numbers: draw j of key
  (round, chain, hop) is output j of the SplitMix64 sequence started from the state
  seed XOR mix(round << 48 | chain << 32 | (hop + 1) << 16).
"""
from __future__ import annotations

import numpy as np

from . import grad as _grad

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
ARMIJO = 1e-4
SIGMA, DELTA, EPS = 0.9, 0.1, 1e-6
MAX_HALVINGS = 20


# ---------------------------------------------------------------- SplitMix64

def splitmix64_mix(z: int) -> int:
    """The output function of SplitMix64."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def splitmix64_sequence(state: int, count: int) -> list:
    """The first ``count`` outputs of SplitMix64 started from ``state``."""
    out = []
    for _ in range(count):
        state = (state + GOLDEN) & MASK
        out.append(splitmix64_mix(state))
    return out


def uniform(seed: int, rnd: int, chain: int, hop: int, j: int) -> float:
    """Draw j (in [0, 1)) of key (round, chain, hop), hop >= -1."""
    key = (rnd << 48) | (chain << 32) | ((hop + 1) << 16)
    state = (seed ^ splitmix64_mix(key)) & MASK
    z = splitmix64_sequence(state, j + 1)[j]
    return (z >> 11) * 2.0 ** -53


# ---------------------------------------------------------------- objective

class Objective:
    """f(x) = -<C> (maximise) or +<C> (minimise) and its gradient, from the FP64 oracle.
    Keyword arguments pick the mixer exactly as ``oracle.grad`` does."""

    def __init__(self, n, table, maximize=True, k=-1, **mixer):
        self.n, self.table, self.k, self.mixer = n, np.asarray(table), k, mixer
        self.sign = -1.0 if maximize else 1.0
        self.calls = 0

    def __call__(self, x):
        self.calls += 1
        E, Nr, g = _grad(self.n, self.table, np.asarray(x, dtype=np.float64), k=self.k, **self.mixer)
        return self.sign * E / Nr, self.sign * g / Nr


# ---------------------------------------------------------------- BFGS

def bfgs(fun, x0, gtol=1e-5, max_iter=100):
    """Local minimisation of fun (returning (f, grad)) from x0: (x, f, accepted steps)."""
    x = np.array(x0, dtype=np.float64)
    D = x.size
    f, g = fun(x)
    H = np.eye(D)
    unscaled = True
    steps = 0

    def done(f, g):
        return np.max(np.abs(g)) <= gtol * max(1.0, abs(f))

    if not np.isfinite(f) or done(f, g) or max_iter <= 0:
        return x, f, steps
    while True:
        d = -H @ g
        gd = g @ d
        if not gd < 0:                       # not a descent direction: steepest descent
            H, unscaled = np.eye(D), True
            d = -g
            gd = g @ d
            if not gd < 0:
                break
        alpha = min(1.0, 1.0 / np.max(np.abs(d)))         # no angle moves more than one radian
        accepted = False
        for _ in range(MAX_HALVINGS + 1):
            xt = x + alpha * d
            ft, gt = fun(xt)
            if np.isfinite(ft):
                armijo = ft <= f + ARMIJO * alpha * gd
                slope = gt @ d
                wolfe = ft <= f + EPS * abs(f) and SIGMA * gd <= slope <= (2 * DELTA - 1) * gd
                if armijo or wolfe:
                    accepted = True
                    break
            alpha *= 0.5
        if not accepted:
            break
        s, y = xt - x, gt - g
        sy = s @ y
        if sy > 1e-10 * np.linalg.norm(s) * np.linalg.norm(y):
            if unscaled:
                H = (sy / (y @ y)) * np.eye(D)
                unscaled = False
            rho = 1.0 / sy
            V = np.eye(D) - rho * np.outer(y, s)
            H = V.T @ H @ V + rho * np.outer(s, s)
        x, f, g = xt, ft, gt
        steps += 1
        if done(f, g) or steps >= max_iter:
            break
    return x, f, steps


# ---------------------------------------------------------------- basinhopping

def basinhopping(fun, seeds, rnd, seed=0, n_hops=10, step=0.5, temperature=1.0, gtol=1e-5, max_iter=100):
    """Chains c start at seeds[c]; returns (best x, best f) over every minimum found, ties to
    the earliest hop, then the lowest chain."""
    seeds = np.asarray(seeds, dtype=np.float64)
    C, D = seeds.shape
    cur, fcur = [], []
    for c in range(C):
        x, f, _ = bfgs(fun, seeds[c], gtol, max_iter)
        cur.append(x)
        fcur.append(f)
    b = int(np.argmin(fcur))                 # first index of the minimum
    bx, bf = cur[b].copy(), fcur[b]
    for h in range(n_hops):
        for c in range(C):
            u = np.array([uniform(seed, rnd, c, h, j) for j in range(D)])
            xm, fm, _ = bfgs(fun, cur[c] + step * (2.0 * u - 1.0), gtol, max_iter)
            if fm < fcur[c]:
                accept = True
            elif temperature > 0 and np.isfinite(fm - fcur[c]):
                accept = uniform(seed, rnd, c, h, D) < np.exp(-(fm - fcur[c]) / temperature)
            else:
                accept = False
            if accept:
                cur[c], fcur[c] = xm, fm
            if fm < bf:
                bx, bf = xm.copy(), fm
    return bx, bf


# ---------------------------------------------------------------- round seeding

def interp(a):
    """INTERP: q values a_1..a_q -> q + 1 values, b_i = ((i-1)/q) a_{i-1} + ((q-i+1)/q) a_i with
    a_0 = a_{q+1} = 0."""
    a = np.asarray(a, dtype=np.float64)
    q = a.size
    ext = np.concatenate([[0.0], a, [0.0]])
    return np.array([((i - 1) / q) * ext[i - 1] + ((q - i + 1) / q) * ext[i] for i in range(1, q + 2)])


def pad_zero_layer(x):
    """(beta_1..beta_q, gamma_1..gamma_q) -> the same with beta_{q+1} = gamma_{q+1} = 0."""
    x = np.asarray(x, dtype=np.float64)
    q = x.size // 2
    return np.concatenate([x[:q], [0.0], x[q:], [0.0]])


def find_angles(fun_for_round, p_max, seed=0, n_chains=8, n_hops=10, step=0.5, temperature=1.0, gtol=1e-5,
                max_iter=100, maximize=True):
    """Iterative rounds 1..p_max; fun_for_round(r) is the objective at r rounds. Round 1: chains
    from uniform angles in [0, 2 pi); round r: chain 0 from the padded round r-1 optimum, the
    others from its INTERP. Returns (list of angle arrays, array of <C>)."""
    sign = -1.0 if maximize else 1.0
    angles, values = [], []
    for r in range(1, p_max + 1):
        D = 2 * r
        if r == 1:
            seeds = np.array([[2 * np.pi * uniform(seed, 1, c, -1, j) for j in range(D)] for c in range(n_chains)])
        else:
            prev = angles[-1]
            itp = np.concatenate([interp(prev[:r - 1]), interp(prev[r - 1:])])
            seeds = np.array([pad_zero_layer(prev) if c == 0 else itp for c in range(n_chains)])
        bx, bf = basinhopping(fun_for_round(r), seeds, r, seed, n_hops, step, temperature, gtol, max_iter)
        angles.append(bx)
        values.append(sign * bf)
    return angles, np.array(values)


def find_angles_random(fun, p, n_restarts, seed=0, gtol=1e-5, max_iter=100, maximize=True):
    """Random local-minima search: BFGS from n_restarts uniform starts in [0, 2 pi)^{2p}.
    Returns (best x, best <C>, <C> of every restart), ties to the lowest restart."""
    sign = -1.0 if maximize else 1.0
    xs, fs = [], []
    for i in range(n_restarts):
        x0 = [2 * np.pi * uniform(seed, p, i, -1, j) for j in range(2 * p)]
        x, f, _ = bfgs(fun, x0, gtol, max_iter)
        xs.append(x)
        fs.append(f)
    b = int(np.argmin(fs))
    return xs[b], sign * fs[b], sign * np.array(fs)
