"""Pins of the oracle's relaxation generator against the paper (CPU only).

* the worked example of the conversion subsection (basis order, representative entries,
  one moment row, two localizing rows, the first equality row and the row count of h_{2,1},
  the five consensus rows) -- tests/golden/worked_example.json;
* the pendulum sizes printed in the abstract and Table 1 (49,500 svec variables,
  47,351 constraints, 30 moment blocks of 55, 60 localizing blocks of 10)
  -- tests/golden/paper_sizes.json;
* the rank-one lifting identities of the refined-certificate subsection: for a feasible
  trajectory z, A(X(z)) = b and <C, X(z)> equals the POP objective.
"""
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _decode_row(sdp, i):
    """Row i as {(block, r, c): coefficient on the matrix entry}, 1-based (r <= c)."""
    out = {}
    for p in range(sdp.rowptr[i], sdp.rowptr[i + 1]):
        col = int(sdp.col[p])
        bk = int(np.searchsorted(sdp.boff, col, side="right") - 1)
        s = col - int(sdp.boff[bk])
        j = int((math.isqrt(8 * s + 1) - 1) // 2)
        r = s - j * (j + 1) // 2
        v = float(sdp.val[p]) * (1.0 if r == j else math.sqrt(2.0))
        out[(bk, r + 1, j + 1)] = v
    return out


def _rows(sdp, kind, clique):
    return [i for i in range(sdp.m) if sdp.rowkind[i] == kind and sdp.rowclique[i] == clique]


@pytest.fixture(scope="module")
def toy(orc):
    dt = 0.1
    return orc.relax(orc.TOY1D, 3, [2.0, dt, 1.0]), dt


def test_basis_order_worked_example(orc, toy):
    sdp, _ = toy
    gold = json.load(open(os.path.join(GOLD, "worked_example.json")))
    x1, u1, x2 = 2.0, 3.0, 5.0
    z = np.array([7.0, 11.0, x1, u1, x2, 13.0, 17.0])
    X, _ = orc.lift(orc.TOY1D, 3, sdp.params, z)
    bk = 2  # block order M_0, L_0, M_1, L_1, ...: the paper's M_2 is our clique 1
    off, n = int(sdp.boff[bk]), int(sdp.bsize[bk])
    first_row = [X[off + j * (j + 1) // 2] / (1.0 if j == 0 else math.sqrt(2.0)) for j in range(n)]
    env = {"x1": x1, "u1": u1, "x2": x2}
    expect = [eval(m.replace("^", "**"), {}, env) if m != "1" else 1.0 for m in gold["basis_M2"]]
    assert np.allclose(first_row, expect, rtol=0, atol=1e-12)


def test_moment_rows_worked_example(orc, toy):
    sdp, _ = toy
    gold = json.load(open(os.path.join(GOLD, "worked_example.json")))
    bk = 2
    rows = [_decode_row(sdp, i) for i in _rows(sdp, orc.ROW_MOMENT, 1)]
    entries = [tuple(e) for e in gold["moment_equal_entries"]]
    # the representative is the first in svec (column-major upper) order: (4,6)
    rep = min(entries, key=lambda rc: (rc[1], rc[0]))
    assert rep == (4, 6)
    for e in entries:
        if e == rep:
            continue
        want = {(bk, *e): 1.0, (bk, *rep): -1.0}
        assert any(r.keys() == want.keys() and all(abs(r[k] - v) < 1e-15 for k, v in want.items())
                   for r in rows), e


def test_localizing_rows_worked_example(orc, toy):
    sdp, _ = toy
    gold = json.load(open(os.path.join(GOLD, "worked_example.json")))
    bM, bL = 2, 3
    rows = [_decode_row(sdp, i) for i in _rows(sdp, orc.ROW_LOCALIZING, 1)]
    for item in gold["localizing"]:
        # L(a,b) = sum coef * M(.)   <=>   L(a,b) - sum coef * M(.) = 0
        want = {(bL, *item["L"]): 1.0}
        for (rc, c) in item["M"]:
            want[(bM, *rc)] = -c
        hits = [r for r in rows if r.keys() == want.keys()]
        assert len(hits) == 1
        assert all(abs(hits[0][k] - v) < 1e-15 for k, v in want.items())


def test_equality_rows_worked_example(orc, toy):
    sdp, dt = toy
    gold = json.load(open(os.path.join(GOLD, "worked_example.json")))
    bM = 2
    eq = _rows(sdp, orc.ROW_EQUALITY, 1)
    assert len(eq) == gold["equality_rows_from_h21"]
    first = _decode_row(sdp, eq[0])
    want = {(bM, *rc): eval(c, {}, {"dt": dt}) for rc, c in gold["equality_first_row"]}
    assert first.keys() == want.keys()
    for k, v in want.items():
        assert abs(first[k] - v) < 1e-15


def test_consensus_rows_worked_example(orc, toy):
    sdp, _ = toy
    gold = json.load(open(os.path.join(GOLD, "worked_example.json")))
    b2, b3 = 2, 4
    rows = [_decode_row(sdp, i) for i in _rows(sdp, orc.ROW_CONSENSUS, 1)]
    pairs = gold["consensus_pairs"]
    assert len(rows) == len(pairs)
    for r, (a, b) in zip(rows, pairs):
        want = {(b2, *a): 1.0, (b3, *b): -1.0}
        assert r.keys() == want.keys()
        assert all(abs(r[k] - v) < 1e-15 for k, v in want.items())


def test_paper_pendulum_sizes(orc):
    gold = json.load(open(os.path.join(GOLD, "paper_sizes.json")))["pendulum"]
    sdp = orc.relax(orc.PAPER_PENDULUM, gold["N"], [0.3, 0.0])
    assert sdp.nsvec == gold["n_svec"]
    assert sdp.m == gold["m"]
    kinds = sdp.bkind
    assert (kinds == 0).sum() == gold["num_M"] and set(sdp.bsize[kinds == 0]) == {gold["size_M"]}
    assert (kinds == 1).sum() == gold["num_L"] and set(sdp.bsize[kinds == 1]) == {gold["size_L"]}


def test_flying_robot_sizes(orc):
    """The paper's flying robot at its horizon: 60 moment blocks of 231 = s(20, 2) (cliques of
    x_k, u_k, x_{k+1} with d_x = 8, d_u = 4) and localizing blocks of 21 = s(20, 1), as in Table 1;
    nine inequalities per clique (four thrust ranges, f_c >= f_c,min, four boxes)."""
    gold = json.load(open(os.path.join(GOLD, "paper_sizes.json")))["flying_robot"]
    sdp = orc.relax(orc.FLYING, gold["N"], [3.0, -2.0, 0.5, 0.5, -0.5, 0.2])
    kinds = sdp.bkind
    assert (kinds == 0).sum() == gold["num_M"] and set(sdp.bsize[kinds == 0]) == {gold["size_M"]}
    assert set(sdp.bsize[kinds == 1]) == {gold["size_L"]}
    assert (kinds == 1).sum() == 9 * gold["N"]
    assert sdp.dx == 8 and sdp.du == 4 and sdp.nclique_vars == 20
    # the paper's m is this relaxation's m plus the rows of the localizing matrices its count has
    # beyond the listed inequalities (tri(21) rows each): the moment, equality, consensus and
    # normalization rows agree with Table 1 exactly
    extra = gold["num_L_paper"] - int((kinds == 1).sum())
    assert sdp.m + extra * (21 * 22 // 2) == gold["m_paper"]


def test_vehicle_landing_sizes(orc):
    """The paper's vehicle landing at its horizon: 50 moment blocks of 190 = s(18, 2) (d_x = 8,
    d_u = 2) and localizing blocks of 19 = s(18, 1), as in Table 1; seven inequalities per clique;
    Table 1's m once the rows of the localizing matrices its count has beyond them are added."""
    gold = json.load(open(os.path.join(GOLD, "paper_sizes.json")))["vehicle_landing"]
    sdp = orc.relax(orc.LANDING, gold["N"], [5.0, 80.0, 0.1, 0.5, -1.0, 0.05])
    kinds = sdp.bkind
    assert (kinds == 0).sum() == gold["num_M"] and set(sdp.bsize[kinds == 0]) == {gold["size_M"]}
    assert set(sdp.bsize[kinds == 1]) == {gold["size_L"]}
    assert (kinds == 1).sum() == 7 * gold["N"]
    extra = gold["num_L_paper"] - int((kinds == 1).sum())
    assert sdp.m + extra * (19 * 20 // 2) == gold["m_paper"]


def test_car_back_in_sizes(orc):
    """The paper's car back-in at its horizon: 30 moment blocks of 190 = s(18, 2) (x_k and x_{k+1}
    of 4, the step's v, w, f_c, f_s and the two separating lines' six coefficients) and localizing
    blocks of 19, as in Table 1; 20 inequalities per clique (16 separations, 4 boxes); Table 1's m
    once the rows of the localizing matrices its count has beyond them are added."""
    gold = json.load(open(os.path.join(GOLD, "paper_sizes.json")))["car_back_in"]
    sdp = orc.relax(orc.BACKIN, gold["N"], [3.0, 4.0, 0.1])
    kinds = sdp.bkind
    assert (kinds == 0).sum() == gold["num_M"] and set(sdp.bsize[kinds == 0]) == {gold["size_M"]}
    assert set(sdp.bsize[kinds == 1]) == {gold["size_L"]}
    assert (kinds == 1).sum() == 20 * gold["N"]
    extra = gold["num_L_paper"] - int((kinds == 1).sum())
    assert sdp.m + extra * (19 * 20 // 2) == gold["m_paper"]


def test_paper_cart_pole_sizes(orc):
    """The paper's cart-pole at its horizon: 30 moment blocks of 105 = s(13, 2) and localizing
    blocks of 14 = s(13, 1), as in Table 1: the second-difference dynamics centred at x_{k+1} put
    (x_k, u_k, x_{k+1}) and a_{k+2}, rs_{k+2} in clique k (d_x = 5, d_u = 1), so consecutive cliques
    share 7 variables.  Modulo tri(14) = 105 every localizing matrix and every equality of degree 2
    adds nothing and an equality of degree 1 adds s(13, 3) = 560 = 35 (mod 105), so with equalities
    of degree <= 2 the normalization, the moment rows and the consensus rows fix m mod 105 up to a
    multiple of 35.  With s(7, 4) = 330 consensus rows per adjacent pair Table 1's m fits (16, as
    here, with a multiple of three linear equalities); with five shared variables (s(5, 4) = 126)
    no count of linear equalities fits (85, 15 or 50).  The paper's localizing count and m
    themselves are not reproduced (three inequalities per clique here)."""
    gold = json.load(open(os.path.join(GOLD, "paper_sizes.json")))["cart_pole"]
    sdp = orc.relax(orc.PAPER_CARTPOLE, gold["N"], [0.1, 0.2, 0.3, 0.5])
    kinds = sdp.bkind
    assert (kinds == 0).sum() == gold["num_M"] and set(sdp.bsize[kinds == 0]) == {gold["size_M"]}
    assert set(sdp.bsize[kinds == 1]) == {gold["size_L"]}
    assert (kinds == 1).sum() == 3 * gold["N"]
    assert sdp.dx == 5 and sdp.du == 1 and sdp.nclique_vars == 13
    assert (sdp.rowkind == orc.ROW_CONSENSUS).sum() == (gold["N"] - 1) * math.comb(7 + 4, 4)
    assert sdp.m % 105 == gold["m_paper"] % 105 == 16
    five = 1 + gold["N"] * (math.comb(15, 2) * (math.comb(15, 2) + 1) // 2 - math.comb(17, 4)) + \
        (gold["N"] - 1) * math.comb(5 + 4, 4)
    assert {(five + 35 * t) % 105 for t in range(3)} == {85, 15, 50}


def test_paper_cart_pole_row_counts(orc):
    """m of the paper's cart-pole reading in closed form: per clique one linear dynamics
    equation and, of degree 2, the pole equation, the rotation r_{k+1} = r_k f_k (2), the sine of
    r_{k+2} (1) and the unit circles of r and f on x_{k+1} (2) and, for k >= 1, on x_k (2); clique
    0 has five initial-state equalities and a_1 from the initial cart velocity."""
    N = 4
    sdp = orc.relax(orc.PAPER_CARTPOLE, N, [0.1, 0.2, 0.3, 0.5])
    d = 13
    s = lambda n: math.comb(d + n, n)
    tri = lambda n: n * (n + 1) // 2
    m = 1 + N * (tri(s(2)) - s(4)) + N * 3 * tri(s(1))
    m += N * (s(3) + 6 * s(2)) + (N - 1) * 2 * s(2) + 6 * s(3)
    m += (N - 1) * math.comb(7 + 4, 4)
    assert sdp.m == m
    assert sdp.nsvec == N * tri(s(2)) + N * 3 * tri(s(1))


def test_paper_cart_pole_step_follows_the_continuous_dynamics(orc):
    """The cart-pole's discrete dynamics (the oracle's step, which the rank-one lifting test ties to
    the relaxation's equality rows) against the continuous model of App. "Cart-Pole" integrated
    to 1e-12: started from the exact a and theta at t = 0 and dt, one step with a constant force
    lands within the integrator's local error of the exact state at 2 dt (here <= 4e-4 in a, 4e-3
    in theta).  A flipped sign of gravity, of the force, of the pole term of the cart equation or
    of the cart term of the pole equation would change the step by far more (each term's size over
    one step is 0.02 to 0.1)."""
    from scipy.integrate import solve_ivp
    m1, m2, l, g, dt = 1.0, 0.3, 0.5, 9.8, 0.1

    def rhs(t, y, u):
        a, th, ad, thd = y
        s, c = np.sin(th), np.cos(th)
        den = m1 + m2 * s * s
        add = (l * m2 * s * thd ** 2 + u + m2 * g * c * s) / den
        thdd = -((l * m2 * s * thd ** 2 + u) * c + (m1 + m2) * g * s) / (l * den)
        return [ad, thd, add, thdd]

    for u, th0, w0, v0 in [(3.0, 0.3, 0.0, 0.0), (-5.0, 1.0, 1.0, 0.5), (0.0, 2.5, -1.0, -0.3), (8.0, -0.7, 2.0, 0.2)]:
        sol = solve_ivp(rhs, [0, 2 * dt], [0, th0, v0, w0], args=(u,), t_eval=[0, dt, 2 * dt], rtol=1e-12,
                        atol=1e-13)
        a, th = sol.y[0], sol.y[1]
        prm = [a[0], (a[1] - a[0]) / dt, th[0], (th[1] - th[0]) / dt]
        z, _ = orc.rollout(orc.PAPER_CARTPOLE, 2, prm, np.full(2, u / 10), 5, 1)
        x2 = z[12:17]  # (a, rc, rs, fc, fs) at step 2
        th2 = th[1] + np.angle((x2[1] + 1j * x2[2]) * np.exp(-1j * th[1]))
        assert abs(x2[0] - a[2]) <= 1e-3
        assert abs(th2 - th[2]) <= 1e-2


def test_flying_robot_row_counts(orc):
    """m of the flying robot from the same closed form as the other families: per clique k >= 1
    three equalities of degree 1 (position updates, f_s update) and eight of degree 2 (velocity
    updates, heading rotation, unit circles of r and f on x_{k+1} and x_k); clique 0 has the eight
    initial-state equalities instead of the two circles on x_0."""
    N = 4
    sdp = orc.relax(orc.FLYING, N, [3.0, -2.0, 0.5, 0.5, -0.5, 0.2])
    d, dx = 20, 8
    s = lambda n: math.comb(d + n, n)
    tri = lambda n: n * (n + 1) // 2
    m = 1 + N * (tri(s(2)) - s(4)) + N * 9 * tri(s(1))
    m += N * (3 * s(3) + 6 * s(2)) + (N - 1) * 2 * s(2) + dx * s(3)
    m += (N - 1) * math.comb(dx + 4, 4)
    assert sdp.m == m


def _binom(n, k):
    return math.comb(n, k)


@pytest.mark.parametrize("fam,N,prm,n_ineq,n_eq_deg", [
    # (family, N, params, inequalities per clique, [(eq degree, count) in clique k >= 1], init count)
    ("PENDULUM", 10, [0.5, 0.0], 1, [(1, 1), (3, 2), (2, 2)]),
    ("CARTPOLE", 6, [0.1, 0.2, 0.5, 0.3], 4, [(1, 1), (3, 1), (4, 1), (3, 2), (2, 2)]),
])
def test_row_counts_closed_form(orc, fam, N, prm, n_ineq, n_eq_deg):
    """m from Prop. 1: tri(s(d,2)) - s(d,4) moment rows, tri(s(d,1)) per localizing matrix,
    s(d, 4 - deg h) per equality, s(d_x, 4) consensus rows per adjacent pair, plus
    d_x initial-state equalities of degree 1 and one normalization row."""
    sdp = orc.relax(getattr(orc, fam), N, prm)
    d, dx = sdp.nclique_vars, sdp.dx
    s = lambda n: _binom(d + n, n)
    tri = lambda n: n * (n + 1) // 2
    eq_k = sum(c * s(4 - dg) for dg, c in n_eq_deg)
    redundant_circle = s(2)  # the unit circle of x_k is repeated in cliques k >= 1
    m = 1 + N * (tri(s(2)) - s(4)) + N * n_ineq * tri(s(1))
    m += N * (eq_k - redundant_circle) + (N - 1) * redundant_circle + dx * s(3)
    m += (N - 1) * _binom(dx + 4, 4)
    assert sdp.m == m
    assert sdp.nsvec == N * tri(s(2)) + N * n_ineq * tri(s(1))


FAMS = [
    ("TOY1D", 3, [2.0, 0.1, 1.0], 0.5),
    ("PENDULUM", 6, [0.5, 0.0], 1.0),
    ("CARTPOLE", 5, [0.1, 0.2, 0.5, 0.3], 1.0),
    ("PAPER_PENDULUM", 4, [0.3, 0.5], 0.5),
    ("CAR", 4, [0, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1], 0.5),
    ("CAR", 4, [1, -1.5, -1.0, 0.3, 1.5, 1.2, 0.0, 0.1], 0.5),
    ("FLYING", 3, [3.0, -2.0, 0.5, 0.5, -0.5, 0.2], 1.0),
    ("LANDING", 3, [5.0, 80.0, 0.1, 0.5, -1.0, 0.05], 1.0),
    ("BACKIN", 3, [3.0, 4.0, 0.1], 1.0),
    ("PAPER_CARTPOLE", 3, [0.1, 0.2, 0.3, 0.5], 1.0),
]


@pytest.mark.parametrize("fam,N,prm,umax", FAMS)
def test_rank_one_lifting(orc, fam, N, prm, umax):
    """A(X(z)) = b and <C,X(z)> = sum_k f_k(z) for feasible rollouts z (refined-certificate
    subsection), and every block of X(z) is PSD when the inequalities hold."""
    f = getattr(orc, fam)
    sdp = orc.relax(f, N, prm)
    rng = np.random.default_rng(7)
    for _ in range(3):
        u = rng.uniform(-umax, umax, N * sdp.du) * 0.5
        z, obj = orc.rollout(f, N, prm, u, sdp.dx, sdp.du)
        X, obj2 = orc.lift(f, N, prm, z)
        assert abs(obj - obj2) <= 1e-12 * (1 + abs(obj))
        res = sdp.A @ X - sdp.b
        assert np.abs(res).max() <= 1e-12 * max(1.0, np.abs(X).max())
        assert abs(sdp.C @ X - obj) <= 1e-11 * (1 + abs(obj))


def test_lifting_detects_infeasible(orc):
    """A trajectory that violates the dynamics leaves equality rows unsatisfied."""
    sdp = orc.relax(orc.PENDULUM, 3, [0.5, 0.0])
    z, _ = orc.rollout(orc.PENDULUM, 3, [0.5, 0.0], np.array([0.2, -0.1, 0.3]), sdp.dx, sdp.du)
    z[5] += 0.05  # perturb omega_1
    X, _ = orc.lift(orc.PENDULUM, 3, [0.5, 0.0], z)
    res = sdp.A @ X - sdp.b
    assert np.abs(res[sdp.rowkind == orc.ROW_EQUALITY]).max() > 1e-3
    assert np.abs(res[sdp.rowkind == orc.ROW_MOMENT]).max() < 1e-12
