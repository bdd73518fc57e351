/*
 * pop.c -- oracle side: polynomials and the trajectory-optimization POP families.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Shares nothing with the HIP path.
 *
 * A trajectory problem (Sec. "Introduction", problem statement) with chain-like sparsity
 * (Def. 1): clique k holds the variables (x_k, u_k, x_{k+1}); every dynamics equality,
 * every set constraint and the stage cost of step k involve only clique k, the terminal
 * cost goes to the last clique.  Variables are rescaled (Sec. "Experiments", general
 * setup) by fixed per-variable factors: original = scale * scaled.  Every equality and
 * inequality polynomial is divided by its largest absolute coefficient.
 */
#include "pop.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ polynomials */

void pl_init(pl_poly *p) { p->n = 0; p->cap = 0; p->t = NULL; }
void pl_free(pl_poly *p) { free(p->t); p->t = NULL; p->n = p->cap = 0; }

static void pl_push(pl_poly *p, const uint8_t *e, double c) {
  if (p->n == p->cap) {
    p->cap = p->cap ? 2 * p->cap : 8;
    p->t = (pl_term *)realloc(p->t, sizeof(pl_term) * (size_t)p->cap);
  }
  memcpy(p->t[p->n].e, e, PL_MAXV);
  p->t[p->n].c = c;
  p->n++;
}

static int term_cmp(const void *a, const void *b) {
  return memcmp(((const pl_term *)a)->e, ((const pl_term *)b)->e, PL_MAXV);
}

/* Merge equal monomials and drop exact zeros. */
void pl_combine(pl_poly *p) {
  if (p->n == 0) return;
  qsort(p->t, (size_t)p->n, sizeof(pl_term), term_cmp);
  int w = 0;
  for (int r = 0; r < p->n; ++r) {
    if (w > 0 && memcmp(p->t[w - 1].e, p->t[r].e, PL_MAXV) == 0) {
      p->t[w - 1].c += p->t[r].c;
    } else {
      p->t[w++] = p->t[r];
    }
  }
  int w2 = 0;
  for (int r = 0; r < w; ++r)
    if (p->t[r].c != 0.0) p->t[w2++] = p->t[r];
  p->n = w2;
}

pl_poly pl_copy(const pl_poly *a) {
  pl_poly p; pl_init(&p);
  for (int i = 0; i < a->n; ++i) pl_push(&p, a->t[i].e, a->t[i].c);
  return p;
}

pl_poly pl_const(double c) {
  pl_poly p; pl_init(&p);
  uint8_t e[PL_MAXV] = {0};
  if (c != 0.0) pl_push(&p, e, c);
  return p;
}

/* c * z_i */
pl_poly pl_var(int i, double c) {
  pl_poly p; pl_init(&p);
  uint8_t e[PL_MAXV] = {0};
  e[i] = 1;
  pl_push(&p, e, c);
  return p;
}

/* a + s*b */
pl_poly pl_axpy(const pl_poly *a, double s, const pl_poly *b) {
  pl_poly p; pl_init(&p);
  for (int i = 0; i < a->n; ++i) pl_push(&p, a->t[i].e, a->t[i].c);
  for (int i = 0; i < b->n; ++i) pl_push(&p, b->t[i].e, s * b->t[i].c);
  pl_combine(&p);
  return p;
}

pl_poly pl_mul(const pl_poly *a, const pl_poly *b) {
  pl_poly p; pl_init(&p);
  for (int i = 0; i < a->n; ++i)
    for (int j = 0; j < b->n; ++j) {
      uint8_t e[PL_MAXV];
      for (int v = 0; v < PL_MAXV; ++v) e[v] = (uint8_t)(a->t[i].e[v] + b->t[j].e[v]);
      pl_push(&p, e, a->t[i].c * b->t[j].c);
    }
  pl_combine(&p);
  return p;
}

int pl_deg(const pl_poly *p) {
  int d = 0;
  for (int i = 0; i < p->n; ++i) {
    int s = 0;
    for (int v = 0; v < PL_MAXV; ++v) s += p->t[i].e[v];
    if (s > d) d = s;
  }
  return d;
}

void pl_normalize(pl_poly *p) {
  double mx = 0.0;
  for (int i = 0; i < p->n; ++i) mx = fmax(mx, fabs(p->t[i].c));
  if (mx > 0.0)
    for (int i = 0; i < p->n; ++i) p->t[i].c /= mx;
}

double pl_eval(const pl_poly *p, const double *z) {
  double s = 0.0;
  for (int i = 0; i < p->n; ++i) {
    double t = p->t[i].c;
    for (int v = 0; v < PL_MAXV; ++v)
      for (int k = 0; k < p->t[i].e[v]; ++k) t *= z[v];
    s += t;
  }
  return s;
}

/* Helpers that consume their arguments, to keep the family code readable. */
static pl_poly add_(pl_poly a, pl_poly b) { pl_poly r = pl_axpy(&a, 1.0, &b); pl_free(&a); pl_free(&b); return r; }
static pl_poly sub_(pl_poly a, pl_poly b) { pl_poly r = pl_axpy(&a, -1.0, &b); pl_free(&a); pl_free(&b); return r; }
static pl_poly mul_(pl_poly a, pl_poly b) { pl_poly r = pl_mul(&a, &b); pl_free(&a); pl_free(&b); return r; }
static pl_poly scl_(double s, pl_poly a) { for (int i = 0; i < a.n; ++i) a.t[i].c *= s; pl_combine(&a); return a; }
static pl_poly sq_(pl_poly a) { pl_poly r = pl_mul(&a, &a); pl_free(&a); return r; }
static pl_poly cst(double c) { return pl_const(c); }

/* ------------------------------------------------------------------ families */

/* Family layout: state / control dimension and the scale of each state and control
 * component (original value = scale * scaled value). */
int fam_layout(int family, const double *prm, int nprm, int *dx, int *du, double *sx, double *su) {
  switch (family) {
    case ORC_TOY1D:
      *dx = 1; *du = 1; sx[0] = 1; su[0] = 1; return 0;
    case ORC_PENDULUM: /* state (rc, rs, omega), control u; omega/8, u/2 */
      *dx = 3; *du = 1; sx[0] = 1; sx[1] = 1; sx[2] = 8; su[0] = 2; return 0;
    case ORC_CARTPOLE: /* state (x, v, rc, rs, omega), control f; v/2, omega/8, f/10 */
      *dx = 5; *du = 1; sx[0] = 1; sx[1] = 2; sx[2] = 1; sx[3] = 1; sx[4] = 8; su[0] = 10;
      return 0;
    case ORC_PAPER_PENDULUM: /* state (rc, rs, fc, fs), control u; u/5 */
      *dx = 4; *du = 1; sx[0] = sx[1] = sx[2] = sx[3] = 1; su[0] = 5; return 0;
    case ORC_CAR: { /* state (rx, ry, rc, rs, v); controls (a, omega) or (a, dtilde, p) */
      if (nprm < 1) return -1;
      int bicycle = prm[0] != 0.0;
      *dx = 5; sx[0] = 3; sx[1] = 3; sx[2] = 1; sx[3] = 1; sx[4] = 2;
      if (bicycle) { *du = 3; su[0] = 2; su[1] = 1; su[2] = 1; }
      else { *du = 2; su[0] = 2; su[1] = 1; }
      return 0;
    }
    case ORC_FLYING: /* state (rx, ry, vx, vy, rc, rs, fc, fs), thrusts u1..u4; r/10, v/10, u/8 */
      *dx = 8; *du = 4;
      sx[0] = sx[1] = sx[2] = sx[3] = 10; sx[4] = sx[5] = sx[6] = sx[7] = 1;
      su[0] = su[1] = su[2] = su[3] = 8;
      return 0;
    case ORC_LANDING: /* state (rx, ry, vx, vy, rc, rs, fc, fs), thrusts u1, u2; rx/100, ry/120, v/20, u/8 */
      *dx = 8; *du = 2;
      sx[0] = 100; sx[1] = 120; sx[2] = sx[3] = 20; sx[4] = sx[5] = sx[6] = sx[7] = 1;
      su[0] = su[1] = 8;
      return 0;
    case ORC_BACKIN: /* state (rx, ry, rc, rs); per step (v, w, fc, fs) and the separating lines
                      * (A1, B1, C1), (A2, B2, C2); r/10, v/4, w/0.5 */
      *dx = 4; *du = 10;
      sx[0] = sx[1] = 10; sx[2] = sx[3] = 1;
      su[0] = 4; su[1] = 0.5;
      for (int i = 2; i < 10; ++i) su[i] = 1;
      return 0;
    case ORC_PAPER_CARTPOLE: /* state (a, rc, rs, fc, fs), force u; a/a_max = a, u/10 */
      *dx = 5; *du = 1; sx[0] = sx[1] = sx[2] = sx[3] = sx[4] = 1; su[0] = 10; return 0;
    default: return -1;
  }
}

/* Lookahead variables: a family whose dynamics span three steps (second differences) has clique
 * k hold, after (x_k, u_k, x_{k+1}), the components lmap[0..dl) of x_{k+2}; clique k+1 holds them
 * in its x_{k+1} part, so consecutive cliques share x_{k+1} and these.  Returns dl. */
int fam_lookahead(int family, int *lmap) {
  if (family == ORC_PAPER_CARTPOLE) { /* a_{k+2} and rs_{k+2} */
    if (lmap) { lmap[0] = 0; lmap[1] = 2; }
    return 2;
  }
  return 0;
}

int orc_lookahead(int family) { return fam_lookahead(family, NULL); }
int orc_lookahead_map(int family, int *lmap) { return fam_lookahead(family, lmap); }

/* Variable in original units: scale * z_i. */
typedef struct { int dx, du; double sx[PL_MAXV], su[PL_MAXV]; int lmap[PL_MAXV]; } lay_t;
static pl_poly X0(const lay_t *L, int i) { return pl_var(i, L->sx[i]); }                 /* x_k     */
static pl_poly U(const lay_t *L, int i) { return pl_var(L->dx + i, L->su[i]); }          /* u_k     */
static pl_poly X1(const lay_t *L, int i) { return pl_var(L->dx + L->du + i, L->sx[i]); } /* x_{k+1} */
/* lookahead j: component lmap[j] of x_{k+2} */
static pl_poly XL(const lay_t *L, int j) { return pl_var(2 * L->dx + L->du + j, L->sx[L->lmap[j]]); }

static void push(pl_list *l, pl_poly p) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 8;
    l->p = (pl_poly *)realloc(l->p, sizeof(pl_poly) * (size_t)l->cap);
  }
  l->p[l->n++] = p;
}

void pl_list_free(pl_list *l) {
  for (int i = 0; i < l->n; ++i) pl_free(&l->p[i]);
  free(l->p);
  l->p = NULL; l->n = l->cap = 0;
}

/* (1 + a^2) c' - (1 - a^2) c + 2 a s  and  (1 + a^2) s' - (1 - a^2) s - 2 a c  with a = rate
 * (a polynomial): the Cayley form of a planar rotation by angle 2*atan(a). */
static void cayley(pl_list *eq, const pl_poly *a, pl_poly c, pl_poly s, pl_poly c1, pl_poly s1) {
  pl_poly a2 = pl_mul(a, a);
  pl_poly one_p = add_(cst(1), pl_copy(&a2)); /* 1 + a^2 */
  pl_poly one_m = sub_(cst(1), pl_copy(&a2)); /* 1 - a^2 */
  pl_poly two_a = scl_(2.0, pl_copy(a));
  pl_poly hc = add_(sub_(pl_mul(&one_p, &c1), pl_mul(&one_m, &c)), pl_mul(&two_a, &s));
  pl_poly hs = sub_(sub_(pl_mul(&one_p, &s1), pl_mul(&one_m, &s)), pl_mul(&two_a, &c));
  push(eq, hc);
  push(eq, hs);
  pl_free(&a2); pl_free(&one_p); pl_free(&one_m); pl_free(&two_a);
  pl_free(&c); pl_free(&s); pl_free(&c1); pl_free(&s1);
}

static pl_poly circle(pl_poly c, pl_poly s) { return sub_(add_(sq_(c), sq_(s)), cst(1)); }

/* Build the constraint and cost polynomials of clique k (variables local to the clique).
 * eq / ineq are appended in the order the relaxation turns them into rows; cost is the
 * stage cost plus, for the last clique, the terminal cost. */
int fam_clique(int family, int N, int k, const double *prm, int nprm, pl_list *eq, pl_list *ineq,
               pl_poly *cost) {
  lay_t L;
  memset(&L, 0, sizeof L);
  if (fam_layout(family, prm, nprm, &L.dx, &L.du, L.sx, L.su)) return -1;
  fam_lookahead(family, L.lmap);
  const int last = (k == N - 1);
  pl_init(cost);

  if (family == ORC_TOY1D) {
    /* xdot = -(1+u)x, direct multiple shooting: x' = x - dt (1+u) x; |u| <= 1;
     * cost u^2 + x^2, terminal P_f x_N^2 (worked example of the paper). */
    if (nprm < 3) return -1;
    const double xinit = prm[0], dt = prm[1], Pf = prm[2];
    if (k == 0) push(eq, sub_(X0(&L, 0), cst(xinit)));
    /* x' + (dt - 1) x + dt u x */
    push(eq, add_(add_(X1(&L, 0), scl_(dt - 1.0, X0(&L, 0))), scl_(dt, mul_(U(&L, 0), X0(&L, 0)))));
    push(ineq, sub_(cst(1), sq_(U(&L, 0))));
    *cost = add_(sq_(U(&L, 0)), sq_(X0(&L, 0)));
    if (last) *cost = add_(*cost, scl_(Pf, sq_(X1(&L, 0))));
  } else if (family == ORC_PENDULUM) {
    /* theta measured from upright: omega' = omega + dt (g/l sin - b/(m l^2) omega + u/(m l^2));
     * (rc, rs) advanced by the Cayley rotation with rate a = dt*omega/2; |u| <= 2;
     * cost (1-rc)^2 + 0.1 omega^2 + 0.01 u^2, terminal P_f [(1-rc)^2 + 0.1 omega^2]. */
    if (nprm < 2) return -1;
    const double m = 1, l = 1, b = 0.1, g = 9.8, dt = 0.1, umax = 2, Pf = 1;
    if (k == 0) {
      push(eq, sub_(X0(&L, 0), cst(cos(prm[0]))));
      push(eq, sub_(X0(&L, 1), cst(sin(prm[0]))));
      push(eq, sub_(X0(&L, 2), cst(prm[1])));
    }
    {
      pl_poly acc = add_(add_(scl_(g / l, X0(&L, 1)), scl_(-b / (m * l * l), X0(&L, 2))),
                         scl_(1.0 / (m * l * l), U(&L, 0)));
      push(eq, sub_(sub_(X1(&L, 2), X0(&L, 2)), scl_(dt, acc)));
    }
    {
      pl_poly a = scl_(dt / 2.0, X0(&L, 2));
      cayley(eq, &a, X0(&L, 0), X0(&L, 1), X1(&L, 0), X1(&L, 1));
      pl_free(&a);
    }
    push(eq, circle(X1(&L, 0), X1(&L, 1)));
    if (k >= 1) push(eq, circle(X0(&L, 0), X0(&L, 1)));
    push(ineq, sub_(cst(umax * umax), sq_(U(&L, 0))));
    *cost = add_(add_(sq_(sub_(cst(1), X0(&L, 0))), scl_(0.1, sq_(X0(&L, 2)))),
                 scl_(0.01, sq_(U(&L, 0))));
    if (last)
      *cost = add_(*cost, scl_(Pf, add_(sq_(sub_(cst(1), X1(&L, 0))), scl_(0.1, sq_(X1(&L, 2))))));
  } else if (family == ORC_CARTPOLE) {
    /* theta from upright (the paper's cart-pole with theta = theta_up + pi), explicit Euler:
     *  (m1 + m2 rs^2)(v' - v) = dt(-l m2 rs w^2 + f + m2 g rc rs)
     *  l (m1 + m2 rs^2)(w' - w) = dt(-l m2 rs rc w^2 + f rc + (m1 + m2) g rs)
     *  x' = x + dt v; Cayley rotation with rate dt*w/2.  |f| <= 10, |x'| <= 1, |v'| <= 4, |w'| <= 16.
     *  Cost: identity on scaled variables, target (0, 0, 1, 0, 0), terminal P_f = 1. */
    if (nprm < 4) return -1;
    const double m1 = 1.0, m2 = 0.3, l = 0.5, g = 9.8, dt = 0.05, fmax_ = 10, xmax = 1, Pf = 1;
    const double vmax = 4, wmax = 16;
    if (k == 0) {
      push(eq, sub_(X0(&L, 0), cst(prm[0])));
      push(eq, sub_(X0(&L, 1), cst(prm[1])));
      push(eq, sub_(X0(&L, 2), cst(cos(prm[2]))));
      push(eq, sub_(X0(&L, 3), cst(sin(prm[2]))));
      push(eq, sub_(X0(&L, 4), cst(prm[3])));
    }
    push(eq, sub_(sub_(X1(&L, 0), X0(&L, 0)), scl_(dt, X0(&L, 1))));
    {
      pl_poly den = add_(cst(m1), scl_(m2, sq_(X0(&L, 3))));
      pl_poly w2 = sq_(X0(&L, 4));
      pl_poly rhs_v = add_(add_(scl_(-l * m2, mul_(X0(&L, 3), pl_copy(&w2))), U(&L, 0)),
                           scl_(m2 * g, mul_(X0(&L, 2), X0(&L, 3))));
      pl_poly hv = sub_(mul_(pl_copy(&den), sub_(X1(&L, 1), X0(&L, 1))), scl_(dt, rhs_v));
      push(eq, hv);
      pl_poly rhs_w = add_(add_(scl_(-l * m2, mul_(mul_(X0(&L, 3), X0(&L, 2)), pl_copy(&w2))),
                                mul_(U(&L, 0), X0(&L, 2))),
                           scl_((m1 + m2) * g, X0(&L, 3)));
      pl_poly hw = sub_(scl_(l, mul_(pl_copy(&den), sub_(X1(&L, 4), X0(&L, 4)))), scl_(dt, rhs_w));
      push(eq, hw);
      pl_free(&den); pl_free(&w2);
    }
    {
      pl_poly a = scl_(dt / 2.0, X0(&L, 4));
      cayley(eq, &a, X0(&L, 2), X0(&L, 3), X1(&L, 2), X1(&L, 3));
      pl_free(&a);
    }
    push(eq, circle(X1(&L, 2), X1(&L, 3)));
    if (k >= 1) push(eq, circle(X0(&L, 2), X0(&L, 3)));
    push(ineq, sub_(cst(fmax_ * fmax_), sq_(U(&L, 0))));
    push(ineq, sub_(cst(xmax * xmax), sq_(X1(&L, 0))));
    /* velocity boxes |v'| <= 4, |w'| <= 16: inactive at the optimum, they bound the moments of
     * the velocities, which nothing else limits (without them the degree-4 moments of w grow
     * without bound along the iteration) */
    push(ineq, sub_(cst(vmax * vmax), sq_(X1(&L, 1))));
    push(ineq, sub_(cst(wmax * wmax), sq_(X1(&L, 4))));
    /* identity weights on the scaled variables: (z_i - target_i)^2 */
    const double tgt[5] = {0, 0, 1, 0, 0};
    for (int i = 0; i < 5; ++i) *cost = add_(*cost, sq_(sub_(pl_var(i, 1.0), cst(tgt[i]))));
    *cost = add_(*cost, sq_(pl_var(L.dx, 1.0)));
    if (last)
      for (int i = 0; i < 5; ++i)
        *cost = add_(*cost, scl_(Pf, sq_(sub_(pl_var(L.dx + L.du + i, 1.0), cst(tgt[i])))));
  } else if (family == ORC_PAPER_PENDULUM) {
    /* Lie-group variational integrator pendulum of the paper's appendix:
     *  m l^2 (fs' - fs)/dt^2 = u - m g l rs - b fs/dt;  r' = r * f (rotation product);
     *  unit circles for r and f;  fc' >= fc_min;  u^2 <= u_max^2. */
    if (nprm < 2) return -1;
    const double m = 1, l = 1, b = 0.1, g = 9.8, dt = 0.1, fcmin = 0.5, umax = 5, Pf = 1;
    if (k == 0) {
      push(eq, sub_(X0(&L, 0), cst(cos(prm[0]))));
      push(eq, sub_(X0(&L, 1), cst(sin(prm[0]))));
      push(eq, sub_(X0(&L, 2), cst(cos(dt * prm[1]))));
      push(eq, sub_(X0(&L, 3), cst(sin(dt * prm[1]))));
    }
    push(eq, add_(add_(scl_(m * l * l / (dt * dt), sub_(X1(&L, 3), X0(&L, 3))), scl_(-1.0, U(&L, 0))),
                  add_(scl_(m * g * l, X0(&L, 1)), scl_(b / dt, X0(&L, 3)))));
    push(eq, sub_(X1(&L, 0), sub_(mul_(X0(&L, 0), X0(&L, 2)), mul_(X0(&L, 1), X0(&L, 3)))));
    push(eq, sub_(X1(&L, 1), add_(mul_(X0(&L, 1), X0(&L, 2)), mul_(X0(&L, 0), X0(&L, 3)))));
    push(eq, circle(X1(&L, 0), X1(&L, 1)));
    push(eq, circle(X1(&L, 2), X1(&L, 3)));
    if (k >= 1) {
      push(eq, circle(X0(&L, 0), X0(&L, 1)));
      push(eq, circle(X0(&L, 2), X0(&L, 3)));
    }
    push(ineq, sub_(X1(&L, 2), cst(fcmin)));
    push(ineq, sub_(cst(umax * umax), sq_(U(&L, 0))));
    const double tgt[4] = {-1, 0, 1, 0};
    for (int i = 0; i < 4; ++i) *cost = add_(*cost, sq_(sub_(pl_var(i, 1.0), cst(tgt[i]))));
    *cost = add_(*cost, sq_(pl_var(L.dx, 1.0)));
    if (last)
      for (int i = 0; i < 4; ++i)
        *cost = add_(*cost, scl_(Pf, sq_(sub_(pl_var(L.dx + L.du + i, 1.0), cst(tgt[i])))));
  } else if (family == ORC_CAR) {
    /* planar car: r' = r + dt v (rc, rs); v' = v + dt a; heading advanced by the Cayley
     * rotation with rate dt*w/2 where w is the turn rate (unicycle) or the lifted yaw rate
     * p = v * dtilde with p - v*dtilde = 0 (bicycle, unit wheelbase).  One circular obstacle
     * of radius 0.5 at o; |rx|,|ry| <= 3, |v| <= 2, |a| <= 2, |w| <= 1.5 or |dtilde| <= 0.6 and
     * |p| <= 1.2.
     * Cost: |r - goal|^2 + v^2 + 0.1 a^2 + 0.1 (w^2 or dtilde^2); terminal P_f = 10. */
    if (nprm < 8) return -1;
    const int bicycle = prm[0] != 0.0;
    const double dt = 0.1, Pf = 10;
    const double sxx = prm[1], syy = prm[2], h0 = prm[3], gx = prm[4], gy = prm[5];
    const double ox = prm[6], oy = prm[7];
    if (k == 0) {
      push(eq, sub_(X0(&L, 0), cst(sxx)));
      push(eq, sub_(X0(&L, 1), cst(syy)));
      push(eq, sub_(X0(&L, 2), cst(cos(h0))));
      push(eq, sub_(X0(&L, 3), cst(sin(h0))));
      push(eq, X0(&L, 4));
    }
    push(eq, sub_(sub_(X1(&L, 0), X0(&L, 0)), scl_(dt, mul_(X0(&L, 4), X0(&L, 2)))));
    push(eq, sub_(sub_(X1(&L, 1), X0(&L, 1)), scl_(dt, mul_(X0(&L, 4), X0(&L, 3)))));
    push(eq, sub_(sub_(X1(&L, 4), X0(&L, 4)), scl_(dt, U(&L, 0))));
    if (bicycle) push(eq, sub_(U(&L, 2), mul_(X0(&L, 4), U(&L, 1))));
    {
      pl_poly a = scl_(dt / 2.0, bicycle ? U(&L, 2) : U(&L, 1));
      cayley(eq, &a, X0(&L, 2), X0(&L, 3), X1(&L, 2), X1(&L, 3));
      pl_free(&a);
    }
    push(eq, circle(X1(&L, 2), X1(&L, 3)));
    if (k >= 1) push(eq, circle(X0(&L, 2), X0(&L, 3)));
    push(ineq, sub_(add_(sq_(sub_(X1(&L, 0), cst(ox))), sq_(sub_(X1(&L, 1), cst(oy)))), cst(0.25)));
    push(ineq, sub_(cst(9), sq_(X1(&L, 0))));
    push(ineq, sub_(cst(9), sq_(X1(&L, 1))));
    push(ineq, sub_(cst(4), sq_(X1(&L, 4))));
    push(ineq, sub_(cst(4), sq_(U(&L, 0))));
    if (bicycle) push(ineq, sub_(cst(0.36), sq_(U(&L, 1))));
    else push(ineq, sub_(cst(2.25), sq_(U(&L, 1))));
    /* |p| <= 1.2 follows from |v| <= 2 and |dtilde| <= 0.6; stated so that the moments of p
     * are bounded too */
    if (bicycle) push(ineq, sub_(cst(1.44), sq_(U(&L, 2))));
    *cost = add_(add_(sq_(sub_(X0(&L, 0), cst(gx))), sq_(sub_(X0(&L, 1), cst(gy)))), sq_(X0(&L, 4)));
    *cost = add_(*cost, scl_(0.1, sq_(U(&L, 0))));
    *cost = add_(*cost, scl_(0.1, sq_(U(&L, 1))));
    if (last)
      *cost = add_(*cost, scl_(Pf, add_(add_(sq_(sub_(X1(&L, 0), cst(gx))), sq_(sub_(X1(&L, 1), cst(gy)))),
                                        sq_(X1(&L, 4)))));
  } else if (family == ORC_FLYING) {
    /* the paper's flying robot (App. "Flying Robot"), Lie-group integrator for the heading:
     *  r' = r + dt v;  v' = v + dt T (rc, rs) with T = u1 - u2 + u3 - u4;
     *  fs' - fs = dt^2 (alpha (u2 - u1) + beta (u3 - u4));  (rc', rs') = (rc, rs) rotated by (fc, fs);
     *  unit circles for r and f;  fc' >= fc_min;  u_i (u_max - u_i) >= 0;  |rx|, |ry|, |vx|, |vy|
     *  within their maxima.  Cost: distance to the rest state at the origin plus |u|^2 (scaled
     *  variables), terminal weight P_f = 10.  Parameters: x0, y0, theta0, vx0, vy0, omega0. */
    if (nprm < 6) return -1;
    const double dt = 0.2, alpha = 0.2, beta = 0.2, fcmin = 0.7, umax = 8, Pf = 10;
    const double rmax = 10, vmax = 10;
    if (k == 0) {
      const double init[8] = {prm[0], prm[1], prm[3], prm[4], cos(prm[2]), sin(prm[2]), cos(dt * prm[5]),
                              sin(dt * prm[5])};
      for (int i = 0; i < 8; ++i) push(eq, sub_(X0(&L, i), cst(init[i])));
    }
    pl_poly T = sub_(add_(sub_(U(&L, 0), U(&L, 1)), U(&L, 2)), U(&L, 3));
    push(eq, sub_(sub_(X1(&L, 0), X0(&L, 0)), scl_(dt, X0(&L, 2))));
    push(eq, sub_(sub_(X1(&L, 1), X0(&L, 1)), scl_(dt, X0(&L, 3))));
    {
      pl_poly T2 = pl_copy(&T);
      push(eq, sub_(sub_(X1(&L, 2), X0(&L, 2)), scl_(dt, mul_(T, X0(&L, 4)))));
      push(eq, sub_(sub_(X1(&L, 3), X0(&L, 3)), scl_(dt, mul_(T2, X0(&L, 5)))));
    }
    push(eq, sub_(sub_(X1(&L, 7), X0(&L, 7)),
                  add_(scl_(dt * dt * alpha, sub_(U(&L, 1), U(&L, 0))), scl_(dt * dt * beta, sub_(U(&L, 2), U(&L, 3))))));
    push(eq, sub_(X1(&L, 4), sub_(mul_(X0(&L, 4), X0(&L, 6)), mul_(X0(&L, 5), X0(&L, 7)))));
    push(eq, sub_(X1(&L, 5), add_(mul_(X0(&L, 5), X0(&L, 6)), mul_(X0(&L, 4), X0(&L, 7)))));
    push(eq, circle(X1(&L, 4), X1(&L, 5)));
    push(eq, circle(X1(&L, 6), X1(&L, 7)));
    if (k >= 1) {
      push(eq, circle(X0(&L, 4), X0(&L, 5)));
      push(eq, circle(X0(&L, 6), X0(&L, 7)));
    }
    for (int i = 0; i < 4; ++i) push(ineq, mul_(U(&L, i), sub_(cst(umax), U(&L, i))));
    push(ineq, sub_(X1(&L, 6), cst(fcmin)));
    push(ineq, sub_(cst(rmax * rmax), sq_(X1(&L, 0))));
    push(ineq, sub_(cst(rmax * rmax), sq_(X1(&L, 1))));
    push(ineq, sub_(cst(vmax * vmax), sq_(X1(&L, 2))));
    push(ineq, sub_(cst(vmax * vmax), sq_(X1(&L, 3))));
    const double tgt[8] = {0, 0, 0, 0, 1, 0, 1, 0};
    for (int i = 0; i < 8; ++i) *cost = add_(*cost, sq_(sub_(pl_var(i, 1.0), cst(tgt[i]))));
    for (int i = 0; i < 4; ++i) *cost = add_(*cost, sq_(pl_var(L.dx + i, 1.0)));
    if (last)
      for (int i = 0; i < 8; ++i)
        *cost = add_(*cost, scl_(Pf, sq_(sub_(pl_var(L.dx + L.du + i, 1.0), cst(tgt[i])))));
  } else if (family == ORC_LANDING) {
    /* the paper's vehicle landing (App. "Vehicle Landing"), Lie-group integrator for the heading:
     *  r' = r + dt v;  m (vx' - vx) = -dt (u1 + u2) rs;  m (vy' - vy) = dt (u1 + u2) rc - dt m g;
     *  I (fs' - fs) = L dt^2 (u2 - u1);  (rc', rs') = (rc, rs) rotated by (fc, fs);  unit circles;
     *  fc' >= fc_min;  u_i (u_max - u_i) >= 0;  |rx| <= rx_max, ry_min <= ry <= ry_max (one
     *  product), |vx|, |vy| <= v_max.  (The appendix writes the gravity term of the vy update
     *  without dt; it is read as the impulse dt m g of one step.)  Cost: distance to rest at
     *  (0, 10) upright plus |u|^2 (scaled variables), terminal weight P_f = 10.  Parameters:
     *  x0, y0, theta0, vx0, vy0, omega0. */
    if (nprm < 6) return -1;
    const double mass = 1, inertia = 50, arm = 5, g = 9.8, dt = 0.2, fcmin = 0.7, umax = 8, Pf = 10;
    const double rxmax = 100, rymin = 10, rymax = 120, vmax = 20;
    if (k == 0) {
      const double init[8] = {prm[0], prm[1], prm[3], prm[4], cos(prm[2]), sin(prm[2]), cos(dt * prm[5]),
                              sin(dt * prm[5])};
      for (int i = 0; i < 8; ++i) push(eq, sub_(X0(&L, i), cst(init[i])));
    }
    pl_poly T = add_(U(&L, 0), U(&L, 1));
    push(eq, sub_(sub_(X1(&L, 0), X0(&L, 0)), scl_(dt, X0(&L, 2))));
    push(eq, sub_(sub_(X1(&L, 1), X0(&L, 1)), scl_(dt, X0(&L, 3))));
    {
      pl_poly T2 = pl_copy(&T);
      push(eq, add_(scl_(mass, sub_(X1(&L, 2), X0(&L, 2))), scl_(dt, mul_(T, X0(&L, 5)))));
      push(eq, add_(sub_(scl_(mass, sub_(X1(&L, 3), X0(&L, 3))), scl_(dt, mul_(T2, X0(&L, 4)))), cst(dt * mass * g)));
    }
    push(eq, sub_(scl_(inertia, sub_(X1(&L, 7), X0(&L, 7))), scl_(arm * dt * dt, sub_(U(&L, 1), U(&L, 0)))));
    push(eq, sub_(X1(&L, 4), sub_(mul_(X0(&L, 4), X0(&L, 6)), mul_(X0(&L, 5), X0(&L, 7)))));
    push(eq, sub_(X1(&L, 5), add_(mul_(X0(&L, 5), X0(&L, 6)), mul_(X0(&L, 4), X0(&L, 7)))));
    push(eq, circle(X1(&L, 4), X1(&L, 5)));
    push(eq, circle(X1(&L, 6), X1(&L, 7)));
    if (k >= 1) {
      push(eq, circle(X0(&L, 4), X0(&L, 5)));
      push(eq, circle(X0(&L, 6), X0(&L, 7)));
    }
    for (int i = 0; i < 2; ++i) push(ineq, mul_(U(&L, i), sub_(cst(umax), U(&L, i))));
    push(ineq, sub_(X1(&L, 6), cst(fcmin)));
    push(ineq, sub_(cst(rxmax * rxmax), sq_(X1(&L, 0))));
    push(ineq, mul_(sub_(X1(&L, 1), cst(rymin)), sub_(cst(rymax), X1(&L, 1))));
    push(ineq, sub_(cst(vmax * vmax), sq_(X1(&L, 2))));
    push(ineq, sub_(cst(vmax * vmax), sq_(X1(&L, 3))));
    const double tgt[8] = {0, 10.0 / 120.0, 0, 0, 1, 0, 1, 0};
    for (int i = 0; i < 8; ++i) *cost = add_(*cost, sq_(sub_(pl_var(i, 1.0), cst(tgt[i]))));
    for (int i = 0; i < 2; ++i) *cost = add_(*cost, sq_(pl_var(L.dx + i, 1.0)));
    if (last)
      for (int i = 0; i < 8; ++i)
        *cost = add_(*cost, scl_(Pf, sq_(sub_(pl_var(L.dx + L.du + i, 1.0), cst(tgt[i])))));
  } else if (family == ORC_BACKIN) {
    /* the paper's car back-in (App. "Car Back-in"): simple car r' = r + dt v (rc, rs), heading
     * rotated by (fc, fs) with fs = dt w - (dt w)^3 / 6; unit circles; no collision of the car (a
     * 6 x 2.5 rectangle at x_{k+1}) with two 8 x 8 squares centred at (6, -4) and (-6, -4), as
     * separating lines A x + B y + C (>= 0 at the car's corners, <= 0 at the square's) with
     * A^2 + B^2 + C^2 = 1; boxes |rx| <= |x0| + 2, |ry| <= 8, |v| <= 4, |w| <= 0.5.  Cost: distance
     * to (0, -3) heading pi/2 plus |(v, w, fc, fs)|^2 (scaled), terminal weight P_f = 10.
     * Parameters: x0, y0, theta0. */
    if (nprm < 3) return -1;
    const double dt = 0.25, Lc = 6, Wc = 2.5, Pf = 10, rymax = 8, vmax = 4, wmax = 0.5;
    const double rxmax = fabs(prm[0]) + 2;
    if (k == 0) {
      const double init[4] = {prm[0], prm[1], cos(prm[2]), sin(prm[2])};
      for (int i = 0; i < 4; ++i) push(eq, sub_(X0(&L, i), cst(init[i])));
    }
    push(eq, sub_(sub_(X1(&L, 0), X0(&L, 0)), scl_(dt, mul_(U(&L, 0), X0(&L, 2)))));
    push(eq, sub_(sub_(X1(&L, 1), X0(&L, 1)), scl_(dt, mul_(U(&L, 0), X0(&L, 3)))));
    {
      pl_poly a = scl_(dt, U(&L, 1));
      pl_poly a3 = mul_(mul_(pl_copy(&a), pl_copy(&a)), pl_copy(&a));
      push(eq, add_(sub_(U(&L, 3), a), scl_(1.0 / 6.0, a3)));
    }
    push(eq, sub_(X1(&L, 2), sub_(mul_(X0(&L, 2), U(&L, 2)), mul_(X0(&L, 3), U(&L, 3)))));
    push(eq, sub_(X1(&L, 3), add_(mul_(X0(&L, 3), U(&L, 2)), mul_(X0(&L, 2), U(&L, 3)))));
    push(eq, circle(X1(&L, 2), X1(&L, 3)));
    push(eq, circle(U(&L, 2), U(&L, 3)));
    if (k >= 1) push(eq, circle(X0(&L, 2), X0(&L, 3)));
    for (int o = 0; o < 2; ++o)
      push(eq, sub_(add_(add_(sq_(U(&L, 4 + 3 * o)), sq_(U(&L, 5 + 3 * o))), sq_(U(&L, 6 + 3 * o))), cst(1)));
    const double cx[2] = {6, -6}, cy[2] = {-4, -4};
    const double sgn[4][2] = {{1, 1}, {-1, 1}, {-1, -1}, {1, -1}};  /* corner i: (+-L/2, +-W/2) */
    for (int o = 0; o < 2; ++o) {
      for (int i = 0; i < 4; ++i) {  /* corner i of the car, in the car's frame (sgn L/2, sgn W/2) */
        const double a = sgn[i][0] * Lc / 2, b = sgn[i][1] * Wc / 2;
        /* xc = x + a c - b s,  yc = y + a s + b c */
        pl_poly xc = add_(X1(&L, 0), sub_(scl_(a, X1(&L, 2)), scl_(b, X1(&L, 3))));
        pl_poly yc = add_(X1(&L, 1), add_(scl_(a, X1(&L, 3)), scl_(b, X1(&L, 2))));
        push(ineq, add_(add_(mul_(U(&L, 4 + 3 * o), xc), mul_(U(&L, 5 + 3 * o), yc)), U(&L, 6 + 3 * o)));
      }
      for (int j = 0; j < 4; ++j) {  /* corner j of square o */
        const double xo = cx[o] + sgn[j][0] * 4, yo = cy[o] + sgn[j][1] * 4;
        push(ineq, scl_(-1.0, add_(add_(scl_(xo, U(&L, 4 + 3 * o)), scl_(yo, U(&L, 5 + 3 * o))), U(&L, 6 + 3 * o))));
      }
    }
    push(ineq, sub_(cst(rxmax * rxmax), sq_(X1(&L, 0))));
    push(ineq, sub_(cst(rymax * rymax), sq_(X1(&L, 1))));
    push(ineq, sub_(cst(vmax * vmax), sq_(U(&L, 0))));
    push(ineq, sub_(cst(wmax * wmax), sq_(U(&L, 1))));
    const double tgt[4] = {0, -0.3, 0, 1};
    for (int i = 0; i < 4; ++i) *cost = add_(*cost, sq_(sub_(pl_var(i, 1.0), cst(tgt[i]))));
    for (int i = 0; i < 4; ++i) *cost = add_(*cost, sq_(pl_var(L.dx + i, 1.0)));
    if (last)
      for (int i = 0; i < 4; ++i)
        *cost = add_(*cost, scl_(Pf, sq_(sub_(pl_var(L.dx + L.du + i, 1.0), cst(tgt[i])))));
  } else if (family == ORC_PAPER_CARTPOLE) {
    /* the paper's cart-pole (App. "Cart-Pole"), Lie-group variational integrator.  State
     * (a, rc, rs, fc, fs): cart position, the pole's angle from the hanging position as a point
     * on the unit circle, and its rotation over one step.  Clique k holds the discrete dynamics
     * centred at step k+1, driven by u_k, with A = a_{k+2} - 2 a_{k+1} + a_k:
     *   (m1 + m2)/dt A + m2 l/dt (rs_{k+2} - 2 rs_{k+1} + rs_k) - dt u_k = 0,
     *   l/dt (fs_{k+1} - fs_k) + A/dt rc_{k+1} + g dt rs_{k+1} = 0,
     * the rotation r_{k+1} = r_k f_k and the sine of r_{k+2} = r_{k+1} f_{k+1}, unit circles,
     * fc >= fc_min, a^2 <= a_max^2, u^2 <= u_max^2.  Initial state: a_0, theta_0 and the step
     * rotation of thetadot_0 fix x_0, adot_0 fixes a_1.  Cost: identity weights on the distance
     * to (a, theta) = (0, pi) at rest and on u (scaled variables), terminal weight P_f. */
    if (nprm < 4) return -1;
    const double m1 = 1.0, m2 = 0.3, l = 0.5, g = 9.8, dt = 0.1, fcmin = 0.5, amax = 1, umax = 10, Pf = 1;
    if (k == 0) {
      push(eq, sub_(X0(&L, 0), cst(prm[0])));
      push(eq, sub_(X0(&L, 1), cst(cos(prm[2]))));
      push(eq, sub_(X0(&L, 2), cst(sin(prm[2]))));
      push(eq, sub_(X0(&L, 3), cst(cos(dt * prm[3]))));
      push(eq, sub_(X0(&L, 4), cst(sin(dt * prm[3]))));
      push(eq, sub_(X1(&L, 0), cst(prm[0] + dt * prm[1])));
    }
    /* second differences of a and rs over (k, k+1, k+2) */
    pl_poly d2a = add_(sub_(XL(&L, 0), scl_(2.0, X1(&L, 0))), X0(&L, 0));
    pl_poly d2s = add_(sub_(XL(&L, 1), scl_(2.0, X1(&L, 2))), X0(&L, 2));
    push(eq, sub_(add_(scl_((m1 + m2) / dt, pl_copy(&d2a)), scl_(m2 * l / dt, d2s)), scl_(dt, U(&L, 0))));
    push(eq, add_(add_(scl_(l / dt, sub_(X1(&L, 4), X0(&L, 4))), scl_(1.0 / dt, mul_(d2a, X1(&L, 1)))),
                  scl_(g * dt, X1(&L, 2))));
    push(eq, sub_(X1(&L, 1), sub_(mul_(X0(&L, 1), X0(&L, 3)), mul_(X0(&L, 2), X0(&L, 4)))));
    push(eq, sub_(X1(&L, 2), add_(mul_(X0(&L, 2), X0(&L, 3)), mul_(X0(&L, 1), X0(&L, 4)))));
    push(eq, sub_(XL(&L, 1), add_(mul_(X1(&L, 2), X1(&L, 3)), mul_(X1(&L, 1), X1(&L, 4)))));
    push(eq, circle(X1(&L, 1), X1(&L, 2)));
    push(eq, circle(X1(&L, 3), X1(&L, 4)));
    if (k >= 1) {
      push(eq, circle(X0(&L, 1), X0(&L, 2)));
      push(eq, circle(X0(&L, 3), X0(&L, 4)));
    }
    push(ineq, sub_(X1(&L, 3), cst(fcmin)));
    push(ineq, sub_(cst(amax * amax), sq_(X1(&L, 0))));
    push(ineq, sub_(cst(umax * umax), sq_(U(&L, 0))));
    const double tgt[5] = {0, -1, 0, 1, 0};
    for (int i = 0; i < 5; ++i) *cost = add_(*cost, sq_(sub_(pl_var(i, 1.0), cst(tgt[i]))));
    *cost = add_(*cost, sq_(pl_var(L.dx, 1.0)));
    if (last)
      for (int i = 0; i < 5; ++i)
        *cost = add_(*cost, scl_(Pf, sq_(sub_(pl_var(L.dx + L.du + i, 1.0), cst(tgt[i])))));
  } else {
    return -1;
  }
  for (int i = 0; i < eq->n; ++i) pl_normalize(&eq->p[i]);
  for (int i = 0; i < ineq->n; ++i) pl_normalize(&ineq->p[i]);
  return 0;
}

/* One explicit step of the dynamics in scaled variables: x1 = F(x0, u).  For the bicycle,
 * the lifted control p is overwritten with v * dtilde so the step is feasible.  aux carries
 * what a family with lookahead needs beyond x (the paper's cart-pole: a_{k+1} in, a_{k+2} out). */
int fam_step(int family, const double *prm, int nprm, const double *x0, double *u, double *x1, double *aux) {
  int dx, du; double sx[PL_MAXV], su[PL_MAXV];
  if (fam_layout(family, prm, nprm, &dx, &du, sx, su)) return -1;
  double X[PL_MAXV], Uo[PL_MAXV], Y[PL_MAXV];
  for (int i = 0; i < dx; ++i) X[i] = x0[i] * sx[i];
  for (int i = 0; i < du; ++i) Uo[i] = u[i] * su[i];
  if (family == ORC_TOY1D) {
    const double dt = prm[1];
    Y[0] = X[0] - dt * (1.0 + Uo[0]) * X[0];
  } else if (family == ORC_PENDULUM) {
    const double m = 1, l = 1, b = 0.1, g = 9.8, dt = 0.1;
    Y[2] = X[2] + dt * (g / l * X[1] - b / (m * l * l) * X[2] + Uo[0] / (m * l * l));
    const double a = dt * X[2] / 2, a2 = a * a;
    Y[0] = ((1 - a2) * X[0] - 2 * a * X[1]) / (1 + a2);
    Y[1] = ((1 - a2) * X[1] + 2 * a * X[0]) / (1 + a2);
  } else if (family == ORC_CARTPOLE) {
    const double m1 = 1.0, m2 = 0.3, l = 0.5, g = 9.8, dt = 0.05;
    const double rc = X[2], rs = X[3], w = X[4], f = Uo[0];
    const double den = m1 + m2 * rs * rs;
    Y[0] = X[0] + dt * X[1];
    Y[1] = X[1] + dt * (-l * m2 * rs * w * w + f + m2 * g * rc * rs) / den;
    Y[4] = w + dt * (-l * m2 * rs * rc * w * w + f * rc + (m1 + m2) * g * rs) / (l * den);
    const double a = dt * w / 2, a2 = a * a;
    Y[2] = ((1 - a2) * rc - 2 * a * rs) / (1 + a2);
    Y[3] = ((1 - a2) * rs + 2 * a * rc) / (1 + a2);
  } else if (family == ORC_PAPER_PENDULUM) {
    const double m = 1, l = 1, b = 0.1, g = 9.8, dt = 0.1;
    Y[3] = X[3] + dt * dt / (m * l * l) * (Uo[0] - m * g * l * X[1] - b / dt * X[3]);
    if (fabs(Y[3]) > 1) return -2;
    Y[2] = sqrt(1 - Y[3] * Y[3]);
    Y[0] = X[0] * X[2] - X[1] * X[3];
    Y[1] = X[1] * X[2] + X[0] * X[3];
  } else if (family == ORC_CAR) {
    const int bicycle = prm[0] != 0.0;
    const double dt = 0.1;
    double w;
    if (bicycle) { Uo[2] = X[4] * Uo[1]; u[2] = Uo[2] / su[2]; w = Uo[2]; }
    else w = Uo[1];
    Y[0] = X[0] + dt * X[4] * X[2];
    Y[1] = X[1] + dt * X[4] * X[3];
    Y[4] = X[4] + dt * Uo[0];
    const double a = dt * w / 2, a2 = a * a;
    Y[2] = ((1 - a2) * X[2] - 2 * a * X[3]) / (1 + a2);
    Y[3] = ((1 - a2) * X[3] + 2 * a * X[2]) / (1 + a2);
  } else if (family == ORC_PAPER_CARTPOLE) {
    /* x_{k+1} = (a_{k+1}, r_k f_k, f_{k+1}); the two dynamics equations centred at k+1 fix the
     * second difference A of a and f_{k+1}: fixed-point iteration on A, a contraction (the
     * factor is at most m2 rc^2 / (m1 + m2) <= 0.24) */
    const double m1 = 1.0, m2 = 0.3, l = 0.5, g = 9.8, dt = 0.1;
    if (!aux) return -1;
    const double a1 = aux[0] * sx[0];
    const double rc1 = X[1] * X[3] - X[2] * X[4], rs1 = X[2] * X[3] + X[1] * X[4];
    double A = 0, fs1 = 0, fc1 = 1;
    for (int it = 0; it < 200; ++it) {
      fs1 = X[4] - (A * rc1 + g * dt * dt * rs1) / l;
      if (fabs(fs1) > 1) return -2;
      fc1 = sqrt(1 - fs1 * fs1);
      const double rs2 = rs1 * fc1 + rc1 * fs1;
      const double An = (dt * dt * Uo[0] - m2 * l * (rs2 - 2 * rs1 + X[2])) / (m1 + m2);
      const int done = fabs(An - A) <= 1e-17;
      A = An;
      if (done) break;
    }
    fs1 = X[4] - (A * rc1 + g * dt * dt * rs1) / l;
    if (fabs(fs1) > 1) return -2;
    fc1 = sqrt(1 - fs1 * fs1);
    Y[0] = a1; Y[1] = rc1; Y[2] = rs1; Y[3] = fc1; Y[4] = fs1;
    aux[0] = (A + 2 * a1 - X[0]) / sx[0];
  } else if (family == ORC_FLYING) {
    const double dt = 0.2, alpha = 0.2, beta = 0.2;
    const double T = Uo[0] - Uo[1] + Uo[2] - Uo[3];
    Y[0] = X[0] + dt * X[2];
    Y[1] = X[1] + dt * X[3];
    Y[2] = X[2] + dt * T * X[4];
    Y[3] = X[3] + dt * T * X[5];
    Y[7] = X[7] + dt * dt * (alpha * (Uo[1] - Uo[0]) + beta * (Uo[2] - Uo[3]));
    if (fabs(Y[7]) > 1) return -2;
    Y[6] = sqrt(1 - Y[7] * Y[7]);
    Y[4] = X[4] * X[6] - X[5] * X[7];
    Y[5] = X[5] * X[6] + X[4] * X[7];
  } else if (family == ORC_LANDING) {
    const double mass = 1, inertia = 50, arm = 5, g = 9.8, dt = 0.2;
    const double T = Uo[0] + Uo[1];
    Y[0] = X[0] + dt * X[2];
    Y[1] = X[1] + dt * X[3];
    Y[2] = X[2] - dt * T * X[5] / mass;
    Y[3] = X[3] + dt * T * X[4] / mass - dt * g;
    Y[7] = X[7] + arm * dt * dt * (Uo[1] - Uo[0]) / inertia;
    if (fabs(Y[7]) > 1) return -2;
    Y[6] = sqrt(1 - Y[7] * Y[7]);
    Y[4] = X[4] * X[6] - X[5] * X[7];
    Y[5] = X[5] * X[6] + X[4] * X[7];
  } else if (family == ORC_BACKIN) {
    /* (fc, fs) from w; each separating line scaled to the unit sphere (or (0, 0, 1)) */
    const double dt = 0.25, a = dt * Uo[1];
    Uo[3] = a - a * a * a / 6;
    if (fabs(Uo[3]) > 1) return -2;
    Uo[2] = sqrt(1 - Uo[3] * Uo[3]);
    for (int o = 0; o < 2; ++o) {
      double *l = Uo + 4 + 3 * o;
      const double nrm = sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
      if (nrm > 0) { l[0] /= nrm; l[1] /= nrm; l[2] /= nrm; } else { l[0] = l[1] = 0; l[2] = 1; }
    }
    for (int i = 2; i < 10; ++i) u[i] = Uo[i] / su[i];
    Y[0] = X[0] + dt * Uo[0] * X[2];
    Y[1] = X[1] + dt * Uo[0] * X[3];
    Y[2] = X[2] * Uo[2] - X[3] * Uo[3];
    Y[3] = X[3] * Uo[2] + X[2] * Uo[3];
  } else {
    return -1;
  }
  for (int i = 0; i < dx; ++i) x1[i] = Y[i] / sx[i];
  return 0;
}

/* Scaled initial state of an instance. */
int fam_init_state(int family, const double *prm, int nprm, double *x0) {
  int dx, du; double sx[PL_MAXV], su[PL_MAXV];
  if (fam_layout(family, prm, nprm, &dx, &du, sx, su)) return -1;
  double X[PL_MAXV];
  /* X holds the initial state in original units */
  if (family == ORC_TOY1D) X[0] = prm[0];
  else if (family == ORC_PENDULUM) { X[0] = cos(prm[0]); X[1] = sin(prm[0]); X[2] = prm[1]; }
  else if (family == ORC_CARTPOLE) {
    X[0] = prm[0]; X[1] = prm[1]; X[2] = cos(prm[2]); X[3] = sin(prm[2]); X[4] = prm[3];
  } else if (family == ORC_PAPER_PENDULUM) {
    X[0] = cos(prm[0]); X[1] = sin(prm[0]); X[2] = cos(0.1 * prm[1]); X[3] = sin(0.1 * prm[1]);
  } else if (family == ORC_CAR) {
    X[0] = prm[1]; X[1] = prm[2]; X[2] = cos(prm[3]); X[3] = sin(prm[3]); X[4] = 0;
  } else if (family == ORC_BACKIN) {
    X[0] = prm[0]; X[1] = prm[1]; X[2] = cos(prm[2]); X[3] = sin(prm[2]);
  } else if (family == ORC_PAPER_CARTPOLE) {
    X[0] = prm[0]; X[1] = cos(prm[2]); X[2] = sin(prm[2]); X[3] = cos(0.1 * prm[3]); X[4] = sin(0.1 * prm[3]);
  } else if (family == ORC_FLYING || family == ORC_LANDING) {
    X[0] = prm[0]; X[1] = prm[1]; X[2] = prm[3]; X[3] = prm[4];
    X[4] = cos(prm[2]); X[5] = sin(prm[2]); X[6] = cos(0.2 * prm[5]); X[7] = sin(0.2 * prm[5]);
  } else return -1;
  for (int i = 0; i < dx; ++i) x0[i] = X[i] / sx[i];
  return 0;
}

/* Bound of the last clique's lookahead variables, which lie past the horizon (0: none beyond the
 * other bounds).  The paper's cart-pole: a_{N+1} has no box, but the dynamics centred at x_N
 * give |a_{N+1}| <= 2|a_N| + |a_{N-1}| + (4 m2 l + dt^2 u_max) / (m1 + m2) (|rs| <= 1). */
double fam_tail_bound(int family, const double *prm, int nprm) {
  if (family == ORC_PAPER_CARTPOLE && nprm >= 4) {
    const double m1 = 1.0, m2 = 0.3, l = 0.5, dt = 0.1, umax = 10;
    const double A = fmax(1.0, fmax(fabs(prm[0]), fabs(prm[0] + dt * prm[1])));
    return 3 * A + (4 * m2 * l + dt * dt * umax) / (m1 + m2);
  }
  return 0.0;
}

/* The step memory of a family with lookahead at the start (the paper's cart-pole: a_1 from the
 * initial cart velocity, scaled). */
int fam_init_aux(int family, const double *prm, int nprm, double *aux) {
  if (family == ORC_PAPER_CARTPOLE) {
    if (nprm < 4) return -1;
    aux[0] = prm[0] + 0.1 * prm[1];
  }
  return 0;
}

/* Bound on every scaled clique variable (x_k, u_k, x_{k+1} order) of a family, from its box
 * constraints, unit circles and initial state; returns -1 when some variable has none (the
 * pendulum's angular rate).  Used for the trace bounds of the certificate. */
int fam_var_bounds(int family, const double *prm, int nprm, double *bnd) {
  int dx, du; double sx[PL_MAXV], su[PL_MAXV];
  if (fam_layout(family, prm, nprm, &dx, &du, sx, su)) return -1;
  double bx[PL_MAXV], bu[PL_MAXV];
  if (family == ORC_TOY1D) {          /* x' = (1 - dt (1 + u)) x with |u| <= 1: |x| <= |x_init| */
    bx[0] = fabs(prm[0]); bu[0] = 1;
  } else if (family == ORC_CARTPOLE) { /* |x'| <= 1, |v'| <= 4, circle, |w'| <= 16, |f| <= 10 */
    bx[0] = fmax(1.0, fabs(prm[0])); bx[1] = fmax(4.0, fabs(prm[1])) / sx[1];
    bx[2] = bx[3] = 1; bx[4] = fmax(16.0, fabs(prm[3])) / sx[4]; bu[0] = 10.0 / su[0];
  } else if (family == ORC_PAPER_PENDULUM) {
    bx[0] = bx[1] = bx[2] = bx[3] = 1; bu[0] = 5.0 / su[0];
  } else if (family == ORC_CAR) {      /* |rx|, |ry| <= 3, circle, |v| <= 2, |a| <= 2, ... */
    bx[0] = fmax(3.0, fabs(prm[1])) / sx[0]; bx[1] = fmax(3.0, fabs(prm[2])) / sx[1];
    bx[2] = bx[3] = 1; bx[4] = 2.0 / sx[4]; bu[0] = 2.0 / su[0];
    if (prm[0] != 0.0) { bu[1] = 0.6; bu[2] = 1.2; } else bu[1] = 1.5;
  } else if (family == ORC_FLYING) {   /* |rx|, |ry|, |vx|, |vy| <= 10, circles, 0 <= u_i <= 8 */
    bx[0] = fmax(10.0, fabs(prm[0])) / sx[0]; bx[1] = fmax(10.0, fabs(prm[1])) / sx[1];
    bx[2] = fmax(10.0, fabs(prm[3])) / sx[2]; bx[3] = fmax(10.0, fabs(prm[4])) / sx[3];
    bx[4] = bx[5] = bx[6] = bx[7] = 1;
    bu[0] = bu[1] = bu[2] = bu[3] = 1;
  } else if (family == ORC_LANDING) {  /* |rx| <= 100, 10 <= ry <= 120, |vx|, |vy| <= 20, circles, 0 <= u <= 8 */
    bx[0] = fmax(100.0, fabs(prm[0])) / sx[0]; bx[1] = fmax(120.0, fabs(prm[1])) / sx[1];
    bx[2] = fmax(20.0, fabs(prm[3])) / sx[2]; bx[3] = fmax(20.0, fabs(prm[4])) / sx[3];
    bx[4] = bx[5] = bx[6] = bx[7] = 1;
    bu[0] = bu[1] = 1;
  } else if (family == ORC_BACKIN) {  /* |rx| <= |x0| + 2, |ry| <= 8 (by 10), circles, |v| <= 4, |w| <= 0.5,
                                        * circle of f, unit spheres of the separating lines */
    bx[0] = (fabs(prm[0]) + 2) / sx[0]; bx[1] = fmax(8.0, fabs(prm[1])) / sx[1];
    bx[2] = bx[3] = 1;
    for (int i = 0; i < 10; ++i) bu[i] = 1;
  } else if (family == ORC_PAPER_CARTPOLE) {
    /* |a_k| <= A = max(a_max, |a_0|, |a_1|) for k <= N (the lookahead a_{k+2} of every clique but
     * the last, see fam_tail_bound), circles, |u| <= 10 (scaled: 1) */
    bx[0] = fmax(1.0, fmax(fabs(prm[0]), fabs(prm[0] + 0.1 * prm[1]))) / sx[0];
    bx[1] = bx[2] = bx[3] = bx[4] = 1;
    bu[0] = 10.0 / su[0];
  } else {
    return -1;
  }
  for (int i = 0; i < dx; ++i) { bnd[i] = bx[i]; bnd[dx + du + i] = bx[i]; }
  for (int i = 0; i < du; ++i) bnd[dx + i] = bu[i];
  return 0;
}
