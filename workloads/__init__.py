"""Seeded synthetic workloads: the random draws that define problem instances.

This module holds no arithmetic of the method (no relaxation, no solver): it only turns a
seed into instance parameters (initial states, goals, horizons, family mix, arrival times)
with SplitMix64 (Steele, Lea and Flood, 2014; a double is the top 53 bits times 2^-53).
Both the product path and the oracle consume its output; neither owns it.

Parameter vectors, per family (angles in radians, original units):
  toy1d    [x_init, dt, P_f]
  pendulum [theta0, omega0]                theta measured from upright, omega0 = 0
  cartpole [x0, v0, theta0, omega0]
  car      [variant, sx, sy, heading0, gx, gy, ox, oy]   variant 0 unicycle-12, 1 bicycle-13
  flying   [x0, y0, theta0, vx0, vy0, omega0]      the paper's flying robot (rest at the origin is the goal)
  landing  [x0, y0, theta0, vx0, vy0, omega0]      the paper's vehicle landing (rest at (0, 10) is the goal)
  backin   [x0, y0, theta0]                        the paper's car back-in (goal (0, -3), heading pi/2)
  paper_cartpole [a0, adot0, theta0, thetadot0]    the paper's cart-pole, theta from hanging (goal upright at a = 0)
"""
from __future__ import annotations

import math

TOY1D, PENDULUM, CARTPOLE, PAPER_PENDULUM, CAR, FLYING, LANDING, BACKIN, PAPER_CARTPOLE = 0, 1, 2, 3, 4, 5, 6, 7, 8
FAMILY_NAMES = {TOY1D: "toy1d", PENDULUM: "pendulum", CARTPOLE: "cartpole",
                PAPER_PENDULUM: "paper_pendulum", CAR: "car", FLYING: "flying",
                LANDING: "landing", BACKIN: "backin", PAPER_CARTPOLE: "paper_cartpole"}
_MASK = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self, lo: float = 0.0, hi: float = 1.0) -> float:
        return lo + (hi - lo) * ((self.next_u64() >> 11) * (1.0 / (1 << 53)))

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1)) % (hi - lo + 1)

    def exponential(self, rate: float) -> float:
        return -math.log(1.0 - self.uniform()) / rate


def _stream(seed: int, tag: int) -> SplitMix64:
    return SplitMix64((seed * 0x100000001B3 + tag * 0x9E3779B1) & _MASK)


def instance_params(family: int, seed: int) -> list:
    """Initial state (and goal / obstacle for the car) of one instance."""
    r = _stream(seed, 17 + family)
    if family == TOY1D:
        return [2.0, 0.1, 1.0]
    if family == PENDULUM:
        return [r.uniform(-math.pi, math.pi), 0.0]
    if family == CARTPOLE:
        return [r.uniform(-0.5, 0.5), r.uniform(-0.5, 0.5), r.uniform(-math.pi, math.pi), r.uniform(-1.0, 1.0)]
    if family == PAPER_PENDULUM:
        return [r.uniform(0.0, math.pi), r.uniform(-5.0, 5.0)]
    if family == CAR:
        variant = seed & 1
        while True:
            sx, sy = r.uniform(-2, 2), r.uniform(-2, 2)
            gx, gy = r.uniform(-2, 2), r.uniform(-2, 2)
            ox, oy = (sx + gx) / 2, (sy + gy) / 2
            if math.hypot(sx - ox, sy - oy) >= 0.6 and math.hypot(gx - ox, gy - oy) >= 0.6:
                break
        return [float(variant), sx, sy, r.uniform(-math.pi, math.pi), gx, gy, ox, oy]
    if family == FLYING:
        return [r.uniform(-5, 5), r.uniform(-5, 5), r.uniform(-math.pi, math.pi), r.uniform(-1, 1), r.uniform(-1, 1),
                r.uniform(-0.5, 0.5)]
    if family == LANDING:
        return [r.uniform(-20, 20), r.uniform(60, 100), r.uniform(-0.3, 0.3), r.uniform(-2, 2), r.uniform(-2, 2),
                r.uniform(-0.2, 0.2)]
    if family == BACKIN:  # above the slot between the two squares, roughly level
        return [r.uniform(2, 5), r.uniform(2, 5), r.uniform(-0.3, 0.3)]
    if family == PAPER_CARTPOLE:  # near the hanging rest state
        return [r.uniform(-0.5, 0.5), r.uniform(-0.5, 0.5), r.uniform(-0.5, 0.5), r.uniform(-1, 1)]
    raise ValueError(family)


# Named configurations: (family, horizon) of the single-instance workloads.
CONFIGS = {
    "C1": (PENDULUM, 10),
    "C2": (CARTPOLE, 30),
    "C3": (CAR, 50),
}


def mixed_batch(seed: int, count: int = 256, nmin: int = 10, nmax: int = 60,
                mix=(1 / 3, 1 / 3, 1 / 3)):
    """A batch of (family, N, params) with families drawn from `mix` over
    (pendulum, cart-pole, car) and horizons uniform on {nmin..nmax}."""
    r = _stream(seed, 101)
    fams = (PENDULUM, CARTPOLE, CAR)
    out = []
    for i in range(count):
        u = r.uniform()
        acc = 0.0
        fam = fams[-1]
        for f, p in zip(fams, mix):
            acc += p
            if u < acc:
                fam = f
                break
        N = r.randint(nmin, nmax)
        out.append((fam, N, instance_params(fam, seed * 100003 + i)))
    return out


def poisson_arrivals(seed: int, rate: float, duration: float, mix=(0.4, 0.4, 0.2), nmin: int = 10,
                     nmax: int = 80):
    """Arrival times (s) and (family, N, params) of a Poisson request stream."""
    r = _stream(seed, 202)
    t = 0.0
    reqs = []
    fams = (PENDULUM, CARTPOLE, CAR)
    i = 0
    while True:
        t += r.exponential(rate)
        if t >= duration:
            break
        u = r.uniform()
        acc = 0.0
        fam = fams[-1]
        for f, p in zip(fams, mix):
            acc += p
            if u < acc:
                fam = f
                break
        N = r.randint(nmin, nmax)
        reqs.append((t, fam, N, instance_params(fam, seed * 1000003 + i)))
        i += 1
    return reqs


def shift_one_clique(block_sizes, svec):
    """Warm start of the next receding-horizon problem: the svec blocks of cliques 1 .. N-1
    moved to cliques 0 .. N-2 and the last clique's blocks repeated (blocks are in clique order,
    each clique's moment block, the largest, first).  Data movement only."""
    import numpy as np
    sizes = [int(n) for n in block_sizes]
    big = max(sizes)
    offs = np.concatenate([[0], np.cumsum([n * (n + 1) // 2 for n in sizes])]).astype(np.int64)
    starts = [k for k, n in enumerate(sizes) if n == big] + [len(sizes)]
    cliques = [svec[offs[a]:offs[b]] for a, b in zip(starts[:-1], starts[1:])]
    return np.concatenate(cliques[1:] + cliques[-1:])
