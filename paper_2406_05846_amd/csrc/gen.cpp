// gen.cpp -- host relaxation generator (see include/strom_gen.h).
//
// Sparse second-order moment relaxation (Prop. 1, relaxation order 2) of a chain-like POP
// (Def. 1) and its PSD-only standard-SDP form ("Faster Conversion to Standard SDP"):
//   * clique k holds (x_k, u_k, x_{k+1}) and, where the dynamics span three steps, some
//     components of x_{k+2} (lookahead); M_k = l([z]_2 [z]_2^T), one localizing matrix
//     l(g [z]_1 [z]_1^T) per inequality g of degree <= 2, l(h [z]_{4 - deg h}) = 0 per
//     equality h, phi_0 = 1;
//   * monomial bases are graded, and descending-lexicographic inside a degree, variables in
//     the order (x_k, u_k, x_{k+1}) -- the order of the worked example's M_2;
//   * a monomial is represented by its first upper-triangle position in svec order; the
//     other positions get a moment row "position - representative";
//   * rows: normalization, then per clique moment / localizing / equality (the initial
//     state first in clique 0) / consensus with the next clique on every monomial of the
//     shared variables (x_{k+1}, then the lookahead); blocks M_0, L_0*, M_1, ...
//   * every equality and inequality polynomial is divided by its largest |coefficient|;
//     variables are used in scaled form (original = scale * scaled).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/strom.h"
#include "../../include/strom_gen.h"

namespace {

// A monomial packs the exponent of variable v into bits [3v, 3v + 3).  Exponents stay below 8
// (total degree <= 4 everywhere), so the product of two monomials is their integer sum; 21
// variables fit 64 bits.
using Mono = uint64_t;
constexpr int kMaxVars = 21;
constexpr int kExpBits = 3;
constexpr Mono kExpMask = 7;

int mono_deg(Mono m) {
  int s = 0;
  for (; m; m >>= kExpBits) s += int(m & kExpMask);
  return s;
}
int mono_exp(Mono m, int v) { return int((m >> (kExpBits * v)) & kExpMask); }
Mono mono_var(int v) { return Mono(1) << (kExpBits * v); }

struct Poly {
  std::map<Mono, double> c;
  Poly() = default;
  explicit Poly(double k) { if (k != 0.0) c[0] = k; }
  static Poly var(int v, double scale) { Poly p; p.c[mono_var(v)] = scale; return p; }
  int degree() const {
    int d = 0;
    for (auto &kv : c) d = std::max(d, mono_deg(kv.first));
    return d;
  }
  void prune() {
    for (auto it = c.begin(); it != c.end();) it = (it->second == 0.0) ? c.erase(it) : std::next(it);
  }
};

Poly operator+(Poly a, const Poly &b) { for (auto &kv : b.c) a.c[kv.first] += kv.second; a.prune(); return a; }
Poly operator-(Poly a, const Poly &b) { for (auto &kv : b.c) a.c[kv.first] -= kv.second; a.prune(); return a; }
Poly operator*(double s, Poly a) { for (auto &kv : a.c) kv.second *= s; a.prune(); return a; }
Poly operator*(const Poly &a, const Poly &b) {
  Poly r;
  for (auto &x : a.c)
    for (auto &y : b.c) r.c[x.first + y.first] += x.second * y.second;
  r.prune();
  return r;
}
Poly operator+(Poly a, double k) { return a + Poly(k); }
Poly operator-(Poly a, double k) { return a - Poly(k); }
Poly operator-(double k, const Poly &a) { return Poly(k) - a; }
Poly operator+(double k, const Poly &a) { return Poly(k) + a; }
Poly sq(const Poly &a) { return a * a; }

void scale_to_unit(Poly &p) {
  double mx = 0.0;
  for (auto &kv : p.c) mx = std::max(mx, std::fabs(kv.second));
  if (mx > 0.0)
    for (auto &kv : p.c) kv.second /= mx;
}

double eval_mono(Mono m, const double *z, int d) {
  double r = 1.0;
  for (int v = 0; v < d; ++v)
    for (int e = mono_exp(m, v); e > 0; --e) r *= z[v];
  return r;
}

// [z]_n over d variables: degree ascending; inside a degree, exponent tuples
// (e_0, e_1, ...) in descending lexicographic order.
void collect_monos(int d, int v, int budget, Mono acc, std::vector<Mono> &all) {
  if (v == d) { all.push_back(acc); return; }
  for (int e = 0; e <= budget; ++e) collect_monos(d, v + 1, budget - e, acc | (Mono(e) << (kExpBits * v)), all);
}

std::vector<Mono> monomial_basis(int d, int n) {
  std::vector<Mono> all;
  collect_monos(d, 0, n, 0, all);  // every exponent tuple of total degree <= n
  std::sort(all.begin(), all.end(), [d](Mono a, Mono b) {
    const int da = mono_deg(a), db = mono_deg(b);
    if (da != db) return da < db;
    for (int v = 0; v < d; ++v) {
      const int ea = mono_exp(a, v), eb = mono_exp(b, v);
      if (ea != eb) return ea > eb;
    }
    return false;
  });
  return all;
}

// ------------------------------------------------------------------------ families

struct Layout {
  int dx = 0, du = 0;
  int dl = 0;                // lookahead variables: components look[0..dl) of x_{k+2}
  int look[kMaxVars] = {0};
  double sx[kMaxVars] = {0}, su[kMaxVars] = {0};
  int nvars() const { return 2 * dx + du + dl; }
  Poly x0(int i) const { return Poly::var(i, sx[i]); }
  Poly u(int i) const { return Poly::var(dx + i, su[i]); }
  Poly x1(int i) const { return Poly::var(dx + du + i, sx[i]); }
  Poly x2(int j) const { return Poly::var(2 * dx + du + j, sx[look[j]]); }  // lookahead j
  Poly zx0(int i) const { return Poly::var(i, 1.0); }       // scaled x_k
  Poly zu(int i) const { return Poly::var(dx + i, 1.0); }   // scaled u_k
  Poly zx1(int i) const { return Poly::var(dx + du + i, 1.0); }
};

struct CliquePolys {
  std::vector<Poly> eq, ineq;
  Poly cost;
};

bool make_layout(int family, const double *p, int np, Layout &L) {
  auto setx = [&](std::initializer_list<double> s) { int i = 0; for (double v : s) L.sx[i++] = v; L.dx = i; };
  auto setu = [&](std::initializer_list<double> s) { int i = 0; for (double v : s) L.su[i++] = v; L.du = i; };
  switch (family) {
    case 0: if (np < 3) return false; setx({1}); setu({1}); return true;
    case 1: if (np < 2) return false; setx({1, 1, 8}); setu({2}); return true;
    case 2: if (np < 4) return false; setx({1, 2, 1, 1, 8}); setu({10}); return true;
    case 3: if (np < 2) return false; setx({1, 1, 1, 1}); setu({5}); return true;
    case 4:
      if (np < 8) return false;
      setx({3, 3, 1, 1, 2});
      if (p[0] != 0.0) setu({2, 1, 1}); else setu({2, 1});
      return true;
    case 5: if (np < 6) return false; setx({10, 10, 10, 10, 1, 1, 1, 1}); setu({8, 8, 8, 8}); return true;
    case 6: if (np < 6) return false; setx({100, 120, 20, 20, 1, 1, 1, 1}); setu({8, 8}); return true;
    case 7: if (np < 3) return false; setx({10, 10, 1, 1}); setu({4, 0.5, 1, 1, 1, 1, 1, 1, 1, 1}); return true;
    case 8:  // (a, rc, rs, fc, fs), force u / 10; a_{k+2} and rs_{k+2} ahead
      if (np < 4) return false;
      setx({1, 1, 1, 1, 1});
      setu({10});
      L.dl = 2;
      L.look[0] = 0;
      L.look[1] = 2;
      return true;
    default: return false;
  }
}

// Cayley form of a planar rotation of (c, s) by 2*atan(a):
//   (1 + a^2) c' - (1 - a^2) c + 2 a s = 0,   (1 + a^2) s' - (1 - a^2) s - 2 a c = 0.
void push_rotation(std::vector<Poly> &eq, const Poly &a, const Poly &c, const Poly &s, const Poly &c1,
                   const Poly &s1) {
  const Poly a2 = sq(a);
  eq.push_back((1.0 + a2) * c1 - (1.0 - a2) * c + 2.0 * (a * s));
  eq.push_back((1.0 + a2) * s1 - (1.0 - a2) * s - 2.0 * (a * c));
}

Poly unit_circle(const Poly &c, const Poly &s) { return sq(c) + sq(s) - 1.0; }

CliquePolys clique_polys(int family, int N, int k, const double *p, const Layout &L) {
  CliquePolys q;
  const bool first = (k == 0), last = (k == N - 1);
  if (family == 0) {  // toy: x' = x - dt (1 + u) x, |u| <= 1, cost u^2 + x^2, terminal P_f x^2
    const double dt = p[1], Pf = p[2];
    if (first) q.eq.push_back(L.x0(0) - p[0]);
    q.eq.push_back(L.x1(0) + (dt - 1.0) * L.x0(0) + dt * (L.u(0) * L.x0(0)));
    q.ineq.push_back(1.0 - sq(L.u(0)));
    q.cost = sq(L.u(0)) + sq(L.x0(0));
    if (last) q.cost = q.cost + Pf * sq(L.x1(0));
  } else if (family == 1) {  // pendulum, theta from upright; Euler on omega, Cayley on (rc, rs)
    const double m = 1, l = 1, b = 0.1, g = 9.8, dt = 0.1, umax = 2, Pf = 1;
    if (first) {
      q.eq.push_back(L.x0(0) - std::cos(p[0]));
      q.eq.push_back(L.x0(1) - std::sin(p[0]));
      q.eq.push_back(L.x0(2) - p[1]);
    }
    const Poly accel = (g / l) * L.x0(1) - (b / (m * l * l)) * L.x0(2) + (1.0 / (m * l * l)) * L.u(0);
    q.eq.push_back(L.x1(2) - L.x0(2) - dt * accel);
    push_rotation(q.eq, (dt / 2) * L.x0(2), L.x0(0), L.x0(1), L.x1(0), L.x1(1));
    q.eq.push_back(unit_circle(L.x1(0), L.x1(1)));
    if (!first) q.eq.push_back(unit_circle(L.x0(0), L.x0(1)));
    q.ineq.push_back(umax * umax - sq(L.u(0)));
    q.cost = sq(1.0 - L.x0(0)) + 0.1 * sq(L.x0(2)) + 0.01 * sq(L.u(0));
    if (last) q.cost = q.cost + Pf * (sq(1.0 - L.x1(0)) + 0.1 * sq(L.x1(2)));
  } else if (family == 2) {  // cart-pole, pole angle from upright
    const double m1 = 1.0, m2 = 0.3, l = 0.5, g = 9.8, dt = 0.05, fmax = 10, xmax = 1, Pf = 1;
    const double vmax = 4, wmax = 16;
    if (first) {
      q.eq.push_back(L.x0(0) - p[0]);
      q.eq.push_back(L.x0(1) - p[1]);
      q.eq.push_back(L.x0(2) - std::cos(p[2]));
      q.eq.push_back(L.x0(3) - std::sin(p[2]));
      q.eq.push_back(L.x0(4) - p[3]);
    }
    const Poly rc = L.x0(2), rs = L.x0(3), w = L.x0(4), f = L.u(0);
    const Poly den = m1 + m2 * sq(rs);
    q.eq.push_back(L.x1(0) - L.x0(0) - dt * L.x0(1));
    q.eq.push_back(den * (L.x1(1) - L.x0(1)) - dt * ((-l * m2) * (rs * sq(w)) + f + (m2 * g) * (rc * rs)));
    q.eq.push_back(l * (den * (L.x1(4) - w)) -
                   dt * ((-l * m2) * (rs * rc * sq(w)) + f * rc + ((m1 + m2) * g) * rs));
    push_rotation(q.eq, (dt / 2) * w, rc, rs, L.x1(2), L.x1(3));
    q.eq.push_back(unit_circle(L.x1(2), L.x1(3)));
    if (!first) q.eq.push_back(unit_circle(rc, rs));
    q.ineq.push_back(fmax * fmax - sq(f));
    q.ineq.push_back(xmax * xmax - sq(L.x1(0)));
    // speed limits (inactive at the optimum) keep every moment of the velocities bounded
    q.ineq.push_back(vmax * vmax - sq(L.x1(1)));
    q.ineq.push_back(wmax * wmax - sq(L.x1(4)));
    const double target[5] = {0, 0, 1, 0, 0};
    for (int i = 0; i < 5; ++i) q.cost = q.cost + sq(L.zx0(i) - target[i]);
    q.cost = q.cost + sq(L.zu(0));
    if (last)
      for (int i = 0; i < 5; ++i) q.cost = q.cost + Pf * sq(L.zx1(i) - target[i]);
  } else if (family == 3) {  // the paper's variational-integrator pendulum (sizes only)
    const double m = 1, l = 1, b = 0.1, g = 9.8, dt = 0.1, fcmin = 0.5, umax = 5, Pf = 1;
    if (first) {
      q.eq.push_back(L.x0(0) - std::cos(p[0]));
      q.eq.push_back(L.x0(1) - std::sin(p[0]));
      q.eq.push_back(L.x0(2) - std::cos(dt * p[1]));
      q.eq.push_back(L.x0(3) - std::sin(dt * p[1]));
    }
    q.eq.push_back((m * l * l / (dt * dt)) * (L.x1(3) - L.x0(3)) - L.u(0) + (m * g * l) * L.x0(1) +
                   (b / dt) * L.x0(3));
    q.eq.push_back(L.x1(0) - (L.x0(0) * L.x0(2) - L.x0(1) * L.x0(3)));
    q.eq.push_back(L.x1(1) - (L.x0(1) * L.x0(2) + L.x0(0) * L.x0(3)));
    q.eq.push_back(unit_circle(L.x1(0), L.x1(1)));
    q.eq.push_back(unit_circle(L.x1(2), L.x1(3)));
    if (!first) {
      q.eq.push_back(unit_circle(L.x0(0), L.x0(1)));
      q.eq.push_back(unit_circle(L.x0(2), L.x0(3)));
    }
    q.ineq.push_back(L.x1(2) - fcmin);
    q.ineq.push_back(umax * umax - sq(L.u(0)));
    const double target[4] = {-1, 0, 1, 0};
    for (int i = 0; i < 4; ++i) q.cost = q.cost + sq(L.zx0(i) - target[i]);
    q.cost = q.cost + sq(L.zu(0));
    if (last)
      for (int i = 0; i < 4; ++i) q.cost = q.cost + Pf * sq(L.zx1(i) - target[i]);
  } else if (family == 5) {  // the paper's flying robot: thrusts u1..u4, Lie-group heading update
    const double dt = 0.2, alpha = 0.2, beta = 0.2, fcmin = 0.7, umax = 8, Pf = 10, rmax = 10, vmax = 10;
    if (first) {
      const double init[8] = {p[0], p[1], p[3], p[4], std::cos(p[2]), std::sin(p[2]), std::cos(dt * p[5]),
                              std::sin(dt * p[5])};
      for (int i = 0; i < 8; ++i) q.eq.push_back(L.x0(i) - init[i]);
    }
    const Poly thrust = L.u(0) - L.u(1) + L.u(2) - L.u(3);
    q.eq.push_back(L.x1(0) - L.x0(0) - dt * L.x0(2));
    q.eq.push_back(L.x1(1) - L.x0(1) - dt * L.x0(3));
    q.eq.push_back(L.x1(2) - L.x0(2) - dt * (thrust * L.x0(4)));
    q.eq.push_back(L.x1(3) - L.x0(3) - dt * (thrust * L.x0(5)));
    q.eq.push_back(L.x1(7) - L.x0(7) - ((dt * dt * alpha) * (L.u(1) - L.u(0)) + (dt * dt * beta) * (L.u(2) - L.u(3))));
    q.eq.push_back(L.x1(4) - (L.x0(4) * L.x0(6) - L.x0(5) * L.x0(7)));
    q.eq.push_back(L.x1(5) - (L.x0(5) * L.x0(6) + L.x0(4) * L.x0(7)));
    q.eq.push_back(unit_circle(L.x1(4), L.x1(5)));
    q.eq.push_back(unit_circle(L.x1(6), L.x1(7)));
    if (!first) {
      q.eq.push_back(unit_circle(L.x0(4), L.x0(5)));
      q.eq.push_back(unit_circle(L.x0(6), L.x0(7)));
    }
    for (int i = 0; i < 4; ++i) q.ineq.push_back(L.u(i) * (umax - L.u(i)));
    q.ineq.push_back(L.x1(6) - fcmin);
    for (int i = 0; i < 2; ++i) q.ineq.push_back(rmax * rmax - sq(L.x1(i)));
    for (int i = 2; i < 4; ++i) q.ineq.push_back(vmax * vmax - sq(L.x1(i)));
    const double target[8] = {0, 0, 0, 0, 1, 0, 1, 0};
    for (int i = 0; i < 8; ++i) q.cost = q.cost + sq(L.zx0(i) - target[i]);
    for (int i = 0; i < 4; ++i) q.cost = q.cost + sq(L.zu(i));
    if (last)
      for (int i = 0; i < 8; ++i) q.cost = q.cost + Pf * sq(L.zx1(i) - target[i]);
  } else if (family == 6) {  // the paper's vehicle landing: two thrusters, Lie-group heading update
    // (the vy update's gravity term is read as the impulse dt m g of one step)
    const double mass = 1, inertia = 50, arm = 5, g = 9.8, dt = 0.2, fcmin = 0.7, umax = 8, Pf = 10;
    const double rxmax = 100, rymin = 10, rymax = 120, vmax = 20;
    if (first) {
      const double init[8] = {p[0], p[1], p[3], p[4], std::cos(p[2]), std::sin(p[2]), std::cos(dt * p[5]),
                              std::sin(dt * p[5])};
      for (int i = 0; i < 8; ++i) q.eq.push_back(L.x0(i) - init[i]);
    }
    const Poly thrust = L.u(0) + L.u(1);
    q.eq.push_back(L.x1(0) - L.x0(0) - dt * L.x0(2));
    q.eq.push_back(L.x1(1) - L.x0(1) - dt * L.x0(3));
    q.eq.push_back(mass * (L.x1(2) - L.x0(2)) + dt * (thrust * L.x0(5)));
    q.eq.push_back(mass * (L.x1(3) - L.x0(3)) - dt * (thrust * L.x0(4)) + dt * mass * g);
    q.eq.push_back(inertia * (L.x1(7) - L.x0(7)) - (arm * dt * dt) * (L.u(1) - L.u(0)));
    q.eq.push_back(L.x1(4) - (L.x0(4) * L.x0(6) - L.x0(5) * L.x0(7)));
    q.eq.push_back(L.x1(5) - (L.x0(5) * L.x0(6) + L.x0(4) * L.x0(7)));
    q.eq.push_back(unit_circle(L.x1(4), L.x1(5)));
    q.eq.push_back(unit_circle(L.x1(6), L.x1(7)));
    if (!first) {
      q.eq.push_back(unit_circle(L.x0(4), L.x0(5)));
      q.eq.push_back(unit_circle(L.x0(6), L.x0(7)));
    }
    for (int i = 0; i < 2; ++i) q.ineq.push_back(L.u(i) * (umax - L.u(i)));
    q.ineq.push_back(L.x1(6) - fcmin);
    q.ineq.push_back(rxmax * rxmax - sq(L.x1(0)));
    q.ineq.push_back((L.x1(1) - rymin) * (rymax - L.x1(1)));
    q.ineq.push_back(vmax * vmax - sq(L.x1(2)));
    q.ineq.push_back(vmax * vmax - sq(L.x1(3)));
    const double target[8] = {0, 10.0 / 120.0, 0, 0, 1, 0, 1, 0};
    for (int i = 0; i < 8; ++i) q.cost = q.cost + sq(L.zx0(i) - target[i]);
    for (int i = 0; i < 2; ++i) q.cost = q.cost + sq(L.zu(i));
    if (last)
      for (int i = 0; i < 8; ++i) q.cost = q.cost + Pf * sq(L.zx1(i) - target[i]);
  } else if (family == 7) {  // the paper's car back-in: two square obstacles, separating lines per step
    // u = (v, w, fc, fs, A1, B1, C1, A2, B2, C2); the car's corners are taken at x_{k+1}
    const double dt = 0.25, Lc = 6, Wc = 2.5, Pf = 10, rymax = 8, vmax = 4, wmax = 0.5;
    const double rxmax = std::fabs(p[0]) + 2;
    if (first) {
      const double init[4] = {p[0], p[1], std::cos(p[2]), std::sin(p[2])};
      for (int i = 0; i < 4; ++i) q.eq.push_back(L.x0(i) - init[i]);
    }
    q.eq.push_back(L.x1(0) - L.x0(0) - dt * (L.u(0) * L.x0(2)));
    q.eq.push_back(L.x1(1) - L.x0(1) - dt * (L.u(0) * L.x0(3)));
    const Poly a = dt * L.u(1);
    q.eq.push_back(L.u(3) - a + (1.0 / 6.0) * (a * a * a));
    q.eq.push_back(L.x1(2) - (L.x0(2) * L.u(2) - L.x0(3) * L.u(3)));
    q.eq.push_back(L.x1(3) - (L.x0(3) * L.u(2) + L.x0(2) * L.u(3)));
    q.eq.push_back(unit_circle(L.x1(2), L.x1(3)));
    q.eq.push_back(unit_circle(L.u(2), L.u(3)));
    if (!first) q.eq.push_back(unit_circle(L.x0(2), L.x0(3)));
    for (int o = 0; o < 2; ++o)
      q.eq.push_back(sq(L.u(4 + 3 * o)) + sq(L.u(5 + 3 * o)) + sq(L.u(6 + 3 * o)) - 1.0);
    const double cx[2] = {6, -6}, cy[2] = {-4, -4};
    const double sgn[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    for (int o = 0; o < 2; ++o) {
      const Poly A = L.u(4 + 3 * o), B = L.u(5 + 3 * o), Cl = L.u(6 + 3 * o);
      for (int i = 0; i < 4; ++i) {  // the car's corner (sgn L/2, sgn W/2) in its own frame
        const double ca = sgn[i][0] * Lc / 2, cb = sgn[i][1] * Wc / 2;
        const Poly xc = L.x1(0) + (ca * L.x1(2) - cb * L.x1(3));
        const Poly yc = L.x1(1) + (ca * L.x1(3) + cb * L.x1(2));
        q.ineq.push_back(A * xc + B * yc + Cl);
      }
      for (int j = 0; j < 4; ++j)  // the square's corner
        q.ineq.push_back(-1.0 * ((cx[o] + sgn[j][0] * 4) * A + (cy[o] + sgn[j][1] * 4) * B + Cl));
    }
    q.ineq.push_back(rxmax * rxmax - sq(L.x1(0)));
    q.ineq.push_back(rymax * rymax - sq(L.x1(1)));
    q.ineq.push_back(vmax * vmax - sq(L.u(0)));
    q.ineq.push_back(wmax * wmax - sq(L.u(1)));
    const double target[4] = {0, -0.3, 0, 1};
    for (int i = 0; i < 4; ++i) q.cost = q.cost + sq(L.zx0(i) - target[i]);
    for (int i = 0; i < 4; ++i) q.cost = q.cost + sq(L.zu(i));
    if (last)
      for (int i = 0; i < 4; ++i) q.cost = q.cost + Pf * sq(L.zx1(i) - target[i]);
  } else if (family == 8) {  // the paper's cart-pole: variational integrator, dynamics centred at x_{k+1}
    // x = (a, rc, rs, fc, fs): r = pole angle from hanging, f = its rotation over a step
    const double m1 = 1.0, m2 = 0.3, l = 0.5, g = 9.8, dt = 0.1, fcmin = 0.5, amax = 1, umax = 10, Pf = 1;
    if (first) {
      const double init[5] = {p[0], std::cos(p[2]), std::sin(p[2]), std::cos(dt * p[3]), std::sin(dt * p[3])};
      for (int i = 0; i < 5; ++i) q.eq.push_back(L.x0(i) - init[i]);
      q.eq.push_back(L.x1(0) - (p[0] + dt * p[1]));  // the cart's initial velocity sets a_1
    }
    const Poly acc = L.x2(0) - 2.0 * L.x1(0) + L.x0(0);   // a_{k+2} - 2 a_{k+1} + a_k
    const Poly sacc = L.x2(1) - 2.0 * L.x1(2) + L.x0(2);  // the same of rs
    q.eq.push_back(((m1 + m2) / dt) * acc + (m2 * l / dt) * sacc - dt * L.u(0));
    q.eq.push_back((l / dt) * (L.x1(4) - L.x0(4)) + (1.0 / dt) * (acc * L.x1(1)) + (g * dt) * L.x1(2));
    q.eq.push_back(L.x1(1) - (L.x0(1) * L.x0(3) - L.x0(2) * L.x0(4)));  // r_{k+1} = r_k f_k
    q.eq.push_back(L.x1(2) - (L.x0(2) * L.x0(3) + L.x0(1) * L.x0(4)));
    q.eq.push_back(L.x2(1) - (L.x1(2) * L.x1(3) + L.x1(1) * L.x1(4)));  // sine of r_{k+1} f_{k+1}
    q.eq.push_back(unit_circle(L.x1(1), L.x1(2)));
    q.eq.push_back(unit_circle(L.x1(3), L.x1(4)));
    if (!first) {
      q.eq.push_back(unit_circle(L.x0(1), L.x0(2)));
      q.eq.push_back(unit_circle(L.x0(3), L.x0(4)));
    }
    q.ineq.push_back(L.x1(3) - fcmin);
    q.ineq.push_back(amax * amax - sq(L.x1(0)));
    q.ineq.push_back(umax * umax - sq(L.u(0)));
    const double target[5] = {0, -1, 0, 1, 0};  // theta = pi, at rest
    for (int i = 0; i < 5; ++i) q.cost = q.cost + sq(L.zx0(i) - target[i]);
    q.cost = q.cost + sq(L.zu(0));
    if (last)
      for (int i = 0; i < 5; ++i) q.cost = q.cost + Pf * sq(L.zx1(i) - target[i]);
  } else {  // planar car with one circular obstacle
    const bool bicycle = p[0] != 0.0;
    const double dt = 0.1, Pf = 10;
    const double gx = p[4], gy = p[5], ox = p[6], oy = p[7];
    if (first) {
      q.eq.push_back(L.x0(0) - p[1]);
      q.eq.push_back(L.x0(1) - p[2]);
      q.eq.push_back(L.x0(2) - std::cos(p[3]));
      q.eq.push_back(L.x0(3) - std::sin(p[3]));
      q.eq.push_back(L.x0(4));
    }
    const Poly v = L.x0(4);
    q.eq.push_back(L.x1(0) - L.x0(0) - dt * (v * L.x0(2)));
    q.eq.push_back(L.x1(1) - L.x0(1) - dt * (v * L.x0(3)));
    q.eq.push_back(L.x1(4) - v - dt * L.u(0));
    if (bicycle) q.eq.push_back(L.u(2) - v * L.u(1));
    push_rotation(q.eq, (dt / 2) * (bicycle ? L.u(2) : L.u(1)), L.x0(2), L.x0(3), L.x1(2), L.x1(3));
    q.eq.push_back(unit_circle(L.x1(2), L.x1(3)));
    if (!first) q.eq.push_back(unit_circle(L.x0(2), L.x0(3)));
    q.ineq.push_back(sq(L.x1(0) - ox) + sq(L.x1(1) - oy) - 0.25);
    q.ineq.push_back(9.0 - sq(L.x1(0)));
    q.ineq.push_back(9.0 - sq(L.x1(1)));
    q.ineq.push_back(4.0 - sq(L.x1(4)));
    q.ineq.push_back(4.0 - sq(L.u(0)));
    q.ineq.push_back(bicycle ? 0.36 - sq(L.u(1)) : 2.25 - sq(L.u(1)));
    if (bicycle) q.ineq.push_back(1.44 - sq(L.u(2)));  // |p| = |v dtilde| <= 1.2, bounds p's moments
    q.cost = sq(L.x0(0) - gx) + sq(L.x0(1) - gy) + sq(v) + 0.1 * sq(L.u(0)) + 0.1 * sq(L.u(1));
    if (last) q.cost = q.cost + Pf * (sq(L.x1(0) - gx) + sq(L.x1(1) - gy) + sq(L.x1(4)));
  }
  for (auto &h : q.eq) scale_to_unit(h);
  for (auto &g : q.ineq) scale_to_unit(g);
  return q;
}

// Bounds on every scaled clique variable implied by the problem (box constraints, unit
// circles, the initial state), state components first, then controls; false when a variable
// has none (the pendulum's angular rate).
bool var_bounds(int family, const double *p, const Layout &L, std::vector<double> &bx, std::vector<double> &bu) {
  bx.assign(size_t(L.dx), 0.0);
  bu.assign(size_t(L.du), 0.0);
  switch (family) {
    case 0: bx = {std::fabs(p[0])}; bu = {1.0}; return true;  // |x| never grows for |u| <= 1
    case 2:  // |x| <= 1, |v| <= 4, unit circle, |w| <= 16, |f| <= 10 (scaled by 1, 2, 1, 1, 8 and 10)
      bx = {std::max(1.0, std::fabs(p[0])), std::max(2.0, std::fabs(p[1]) / 2), 1.0, 1.0,
            std::max(2.0, std::fabs(p[3]) / 8)};
      bu = {1.0};
      return true;
    case 3: bx = {1.0, 1.0, 1.0, 1.0}; bu = {1.0}; return true;  // unit circles, |u| <= 5 (scaled by 5)
    case 4:  // |rx|, |ry| <= 3, unit circle, |v| <= 2, |a| <= 2; |w| <= 1.5 or |dtilde| <= 0.6 and |p| <= 1.2
      bx = {std::max(1.0, std::fabs(p[1]) / 3), std::max(1.0, std::fabs(p[2]) / 3), 1.0, 1.0, 1.0};
      if (p[0] != 0.0) bu = {1.0, 0.6, 1.2}; else bu = {1.0, 1.5};
      return true;
    case 5:  // |rx|, |ry|, |vx|, |vy| <= 10 (scaled by 10), circles, 0 <= u_i <= 8 (scaled by 8)
      bx = {std::max(1.0, std::fabs(p[0]) / 10), std::max(1.0, std::fabs(p[1]) / 10),
            std::max(1.0, std::fabs(p[3]) / 10), std::max(1.0, std::fabs(p[4]) / 10), 1.0, 1.0, 1.0, 1.0};
      bu = {1.0, 1.0, 1.0, 1.0};
      return true;
    case 6:  // |rx| <= 100, 10 <= ry <= 120, |vx|, |vy| <= 20 (scaled by 100, 120, 20, 20), circles, 0 <= u <= 8
      bx = {std::max(1.0, std::fabs(p[0]) / 100), std::max(1.0, std::fabs(p[1]) / 120),
            std::max(1.0, std::fabs(p[3]) / 20), std::max(1.0, std::fabs(p[4]) / 20), 1.0, 1.0, 1.0, 1.0};
      bu = {1.0, 1.0};
      return true;
    case 7:  // |rx| <= |x0| + 2, |ry| <= 8 (scaled by 10), circles; |v| <= 4, |w| <= 0.5, circle, unit spheres
      bx = {(std::fabs(p[0]) + 2) / 10, std::max(8.0, std::fabs(p[1])) / 10, 1.0, 1.0};
      bu.assign(10, 1.0);
      return true;
    case 8:  // |a| <= A for a_0..a_N (see tail_bound for the last clique's a_{N+1}); circles; |u| <= 10
      bx = {std::max(1.0, std::max(std::fabs(p[0]), std::fabs(p[0] + 0.1 * p[1]))), 1.0, 1.0, 1.0, 1.0};
      bu = {1.0};
      return true;
    default: return false;
  }
}

// Bound of the last clique's variables past the horizon (0: none beyond var_bounds): the
// paper's cart-pole holds a_{N+1}, which only its dynamics centred at x_N bound:
// |a_{N+1}| <= 2|a_N| + |a_{N-1}| + (4 m2 l + dt^2 u_max)/(m1 + m2).
double tail_bound(int family, const double *p) {
  if (family != 8) return 0.0;
  const double A = std::max(1.0, std::max(std::fabs(p[0]), std::fabs(p[0] + 0.1 * p[1])));
  return 3 * A + (4 * 0.3 * 0.5 + 0.1 * 0.1 * 10) / (1.0 + 0.3);
}

// An upper bound of g over the box |z_v| <= R: exact for the terms of one variable of degree
// <= 2 (each variable's together), |c| R^deg for every other term (products of two variables in
// the car back-in's separation inequalities), the latter summed in ascending order.
bool box_max(const Poly &g, double R, double &out) {
  std::map<int, std::pair<double, double>> ab;  // variable -> (coefficient of z^2, of z)
  std::vector<double> other;
  double c = 0.0;
  for (auto &t : g.c) {
    if (t.first == 0) { c += t.second; continue; }
    int var = -1, e = 0, nv = 0;
    for (int v = 0; v < kMaxVars; ++v)
      if (mono_exp(t.first, v)) {
        var = v;
        e = mono_exp(t.first, v);
        ++nv;
      }
    if (nv == 1 && e == 2) ab[var].first += t.second;
    else if (nv == 1 && e == 1) ab[var].second += t.second;
    else {
      double m = std::fabs(t.second);
      for (int q = mono_deg(t.first); q > 0; --q) m *= R;
      other.push_back(m);
    }
  }
  for (auto &kv : ab) {
    const double a = kv.second.first, b = kv.second.second;
    double m = std::max(a * R * R + b * R, a * R * R - b * R);
    if (a != 0.0) {
      const double t = -b / (2 * a);
      if (std::fabs(t) <= R) m = std::max(m, a * t * t + b * t);
    }
    c += m;
  }
  std::sort(other.begin(), other.end());
  double so = 0.0;
  for (double v : other) so += v;
  out = c + so;
  return true;
}

}  // namespace

// ------------------------------------------------------------------------ relaxation

struct strom_gen_sdp {
  std::vector<int32_t> block_sizes;
  std::vector<int64_t> rowptr{0};
  std::vector<int32_t> col;
  std::vector<double> val;
  std::vector<double> b;
  std::vector<double> C;
  std::vector<int32_t> kind;
  int64_t nsvec = 0;
  std::vector<double> trace_bound;  // R_beta per block (empty: some variable is unbounded)
};

namespace {

struct RowWriter {
  strom_gen_sdp &out;
  std::vector<std::pair<int32_t, double>> cur;
  void put(int64_t block_off, int i, int j, double coef) {
    if (i > j) std::swap(i, j);
    const double sv = (i == j) ? coef : coef / std::sqrt(2.0);  // undo the svec sqrt(2)
    cur.emplace_back(int32_t(block_off + int64_t(j) * (j + 1) / 2 + i), sv);
  }
  void close(int kind, double rhs) {
    std::sort(cur.begin(), cur.end());
    for (size_t a = 0; a < cur.size();) {
      size_t e = a;
      double s = 0.0;
      while (e < cur.size() && cur[e].first == cur[a].first) s += cur[e++].second;
      if (s != 0.0) { out.col.push_back(cur[a].first); out.val.push_back(s); }
      a = e;
    }
    cur.clear();
    out.rowptr.push_back(int64_t(out.col.size()));
    out.b.push_back(rhs);
    out.kind.push_back(kind);
  }
};

}  // namespace

extern "C" int strom_gen_build(int family, int N, const double *params, int nparams,
                               strom_gen_sdp **out) {
  if (!out) return STROM_E_INVAL;
  *out = nullptr;
  Layout L;
  if (N < 1 || !params || !make_layout(family, params, nparams, L)) return STROM_E_INVAL;
  const int d = L.nvars();
  if (d > kMaxVars) return STROM_E_INVAL;

  const std::vector<Mono> B2 = monomial_basis(d, 2), B1 = monomial_basis(d, 1);
  const int nM = int(B2.size()), n1 = int(B1.size());
  // representative (first svec position) of every monomial of M
  std::unordered_map<Mono, std::pair<int, int>> rep;
  rep.reserve(size_t(nM) * nM);
  for (int j = 0; j < nM; ++j)
    for (int i = 0; i <= j; ++i) rep.emplace(B2[size_t(i)] + B2[size_t(j)], std::make_pair(i, j));

  std::vector<CliquePolys> cl;
  cl.reserve(size_t(N));
  for (int k = 0; k < N; ++k) cl.push_back(clique_polys(family, N, k, params, L));
  for (auto &q : cl) {
    for (auto &h : q.eq) if (h.degree() > 4) return STROM_E_INVAL;
    for (auto &g : q.ineq) if (g.degree() < 1 || g.degree() > 2) return STROM_E_INVAL;
    if (q.cost.degree() > 4) return STROM_E_INVAL;
  }

  auto *S = new strom_gen_sdp();
  std::vector<int64_t> offM(static_cast<size_t>(N));
  std::vector<std::vector<int64_t>> offL(static_cast<size_t>(N));
  int64_t off = 0;
  for (int k = 0; k < N; ++k) {
    offM[size_t(k)] = off;
    S->block_sizes.push_back(nM);
    off += int64_t(nM) * (nM + 1) / 2;
    for (size_t gi = 0; gi < cl[size_t(k)].ineq.size(); ++gi) {
      offL[size_t(k)].push_back(off);
      S->block_sizes.push_back(n1);
      off += int64_t(n1) * (n1 + 1) / 2;
    }
  }
  S->nsvec = off;
  S->C.assign(size_t(off), 0.0);
  // Trace bounds of the rank-one liftings (App. "Existence of R_beta"): with |z_v| <= R_k on the
  // clique, every monomial of degree <= t is at most max(1, R_k)^t in size, so
  // tr M_k(z) = ||[z]_2||^2 <= s(d, 2) max(1, R_k)^4 and tr L_{k,i}(z) <= max_box g * s(d, 1) max(1, R_k)^2.
  {
    std::vector<double> bx, bu;
    if (var_bounds(family, params, L, bx, bu)) {
      double R0 = 0.0;
      for (double v : bx) R0 = std::max(R0, v);
      for (double v : bu) R0 = std::max(R0, v);
      bool ok = true;
      for (int k = 0; k < N && ok; ++k) {
        const double Rk = k == N - 1 ? std::max(R0, tail_bound(family, params)) : R0;  // past the horizon
        const double r1 = std::max(1.0, Rk);
        S->trace_bound.push_back(double(nM) * r1 * r1 * r1 * r1);
        for (const Poly &g : cl[size_t(k)].ineq) {
          double gm = 0.0;
          ok = ok && box_max(g, Rk, gm);
          S->trace_bound.push_back(std::max(0.0, gm) * double(n1) * r1 * r1);
        }
      }
      if (!ok) S->trace_bound.clear();
    }
  }

  RowWriter W{*S, {}};
  auto put_rep = [&](int k, Mono mono, double coef) {
    const auto &ij = rep.at(mono);
    W.put(offM[size_t(k)], ij.first, ij.second, coef);
  };

  W.put(offM[0], 0, 0, 1.0);  // phi_0 = M_0(1,1) = 1
  W.close(0, 1.0);
  // the variables clique k shares with clique k+1: x_{k+1} and the lookahead, the last dx + dl of
  // clique k; in clique k+1, x_{k+1} comes first and the lookahead sits in its x_{k+2} part
  const int nshared = L.dx + L.dl;
  const std::vector<Mono> Bshared = monomial_basis(nshared, 4);
  auto in_next = [&](Mono a) {
    Mono r = 0;
    for (int v = 0; v < nshared; ++v) {
      const int pos = v < L.dx ? v : L.dx + L.du + L.look[v - L.dx];
      r += Mono(mono_exp(a, v)) << (kExpBits * pos);
    }
    return r;
  };
  for (int k = 0; k < N; ++k) {
    const CliquePolys &q = cl[size_t(k)];
    for (int j = 0; j < nM; ++j)  // moment rows
      for (int i = 0; i <= j; ++i) {
        const auto &r = rep.at(B2[size_t(i)] + B2[size_t(j)]);
        if (r.first == i && r.second == j) continue;
        W.put(offM[size_t(k)], i, j, 1.0);
        W.put(offM[size_t(k)], r.first, r.second, -1.0);
        W.close(1, 0.0);
      }
    for (size_t gi = 0; gi < q.ineq.size(); ++gi)  // localizing rows
      for (int bcol = 0; bcol < n1; ++bcol)
        for (int a = 0; a <= bcol; ++a) {
          W.put(offL[size_t(k)][gi], a, bcol, 1.0);
          for (auto &t : q.ineq[gi].c) put_rep(k, B1[size_t(a)] + B1[size_t(bcol)] + t.first, -t.second);
          W.close(2, 0.0);
        }
    for (const Poly &h : q.eq) {  // equality rows
      for (Mono mult : monomial_basis(d, 4 - h.degree())) {
        for (auto &t : h.c) put_rep(k, mult + t.first, t.second);
        W.close(3, 0.0);
      }
    }
    if (k + 1 < N) {  // consensus rows on the monomials of the shared variables
      const int shift = kExpBits * (L.dx + L.du);
      for (Mono a : Bshared) {
        put_rep(k, a << shift, 1.0);
        put_rep(k + 1, in_next(a), -1.0);
        W.close(4, 0.0);
      }
    }
    for (auto &t : q.cost.c) {  // objective on the representatives
      const auto &ij = rep.at(t.first);
      const int64_t s = offM[size_t(k)] + int64_t(ij.second) * (ij.second + 1) / 2 + ij.first;
      S->C[size_t(s)] += (ij.first == ij.second) ? t.second : t.second / std::sqrt(2.0);
    }
  }
  *out = S;
  return 0;
}

extern "C" int strom_gen_sizes(const strom_gen_sdp *g, int32_t *nblocks, int32_t *m, int64_t *nnz,
                               int64_t *n_svec) {
  if (!g) return STROM_E_INVAL;
  if (nblocks) *nblocks = int32_t(g->block_sizes.size());
  if (m) *m = int32_t(g->b.size());
  if (nnz) *nnz = int64_t(g->col.size());
  if (n_svec) *n_svec = g->nsvec;
  return 0;
}

extern "C" int strom_gen_export(const strom_gen_sdp *g, int32_t *block_sizes, int64_t *rowptr,
                                int32_t *col, double *val, double *b, double *C_svec, int32_t *row_kind) {
  if (!g || !block_sizes || !rowptr || !col || !val || !b || !C_svec) return STROM_E_INVAL;
  std::memcpy(block_sizes, g->block_sizes.data(), g->block_sizes.size() * sizeof(int32_t));
  std::memcpy(rowptr, g->rowptr.data(), g->rowptr.size() * sizeof(int64_t));
  std::memcpy(col, g->col.data(), g->col.size() * sizeof(int32_t));
  std::memcpy(val, g->val.data(), g->val.size() * sizeof(double));
  std::memcpy(b, g->b.data(), g->b.size() * sizeof(double));
  std::memcpy(C_svec, g->C.data(), g->C.size() * sizeof(double));
  if (row_kind) std::memcpy(row_kind, g->kind.data(), g->kind.size() * sizeof(int32_t));
  return 0;
}

extern "C" void strom_gen_free(strom_gen_sdp *g) { delete g; }

extern "C" int strom_gen_trace_bounds(const strom_gen_sdp *g, double *R_beta) {
  if (!g || !R_beta) return STROM_E_INVAL;
  if (g->trace_bound.empty()) return STROM_E_INVAL;
  std::memcpy(R_beta, g->trace_bound.data(), g->trace_bound.size() * sizeof(double));
  return 0;
}
