/*
 * relax.c -- oracle side: sparse second-order moment relaxation of a chain-like POP and its
 * conversion to a PSD-only multi-block SDP.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Shares nothing with the HIP path.
 *
 * Follows the paper's Sec. "Sparse Moment Relaxation":
 *   - relaxation order kappa = 2 (Prop. 1); the moment matrix of clique k is
 *     M_k = l_phi([z(I_k)]_2 [z(I_k)]_2^T), every inequality g gives the localizing matrix
 *     L_{k,i} = l_phi(g [z]_{2-ceil(deg g/2)} [z]^T), every equality h gives the localizing
 *     vector l_phi(h [z]_{4 - deg h}) = 0, and phi_0 = 1;
 *   - the conversion to the standard form min <C,X> s.t. A(X) = b, X PSD (the
 *     "Faster Conversion to Standard SDP" subsection) with the four row types of the worked
 *     example: moment (repeated monomials inside M_k), localizing (entries of L_{k,i} as
 *     combinations of entries of M_k), equality, consensus (monomials shared by M_k and
 *     M_{k+1}), plus the normalization phi_0 = 1.
 *
 * Conventions (each reproduces the indices printed in the worked example):
 *   - monomial basis [z]_n: graded by degree, inside a degree the exponent tuples in
 *     descending lexicographic order, variables in the order (x_k, u_k, x_{k+1}), then, for a
 *     family whose dynamics span three steps, its lookahead components of x_{k+2};
 *   - svec: column-major upper triangle, off-diagonal entries times sqrt(2);
 *   - the representative entry of a monomial in M_k is its first occurrence in svec order;
 *     localizing, equality, consensus rows and the objective refer to representatives;
 *   - a moment row is "occurrence minus representative" for each non-representative upper
 *     entry, in svec order;
 *   - row order: normalization first, then per clique: moment, localizing, equality (the
 *     initial-state equalities first in clique 0), consensus with the next clique;
 *   - block order: M_0, L_{0,*}, M_1, L_{1,*}, ...
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "pop.h"

typedef uint8_t mono_t[PL_MAXV];

/* ---------------------------------------------------------------- monomial bases */

static void enum_deg(int d, int deg, int pos, uint8_t *cur, mono_t *out, int *cnt) {
  if (pos == d - 1) {
    cur[pos] = (uint8_t)deg;
    if (out) memcpy(out[*cnt], cur, PL_MAXV);
    (*cnt)++;
    return;
  }
  for (int e = deg; e >= 0; --e) {
    cur[pos] = (uint8_t)e;
    enum_deg(d, deg - e, pos + 1, cur, out, cnt);
  }
  cur[pos] = 0;
}

/* [z]_n for d variables; returns the count and allocates *out. */
static int basis(int d, int n, mono_t **out) {
  uint8_t cur[PL_MAXV];
  int cnt = 0;
  memset(cur, 0, sizeof cur);
  for (int deg = 0; deg <= n; ++deg) enum_deg(d, deg, 0, cur, NULL, &cnt);
  *out = (mono_t *)calloc((size_t)cnt, sizeof(mono_t));
  int c2 = 0;
  memset(cur, 0, sizeof cur);
  for (int deg = 0; deg <= n; ++deg) enum_deg(d, deg, 0, cur, *out, &c2);
  return cnt;
}

/* Key of a monomial: exponent of variable v in bits [3v, 3v + 3).  Every monomial here has total
 * degree <= 4, so each exponent fits three bits and the key is unique. */
static uint64_t mkey(const uint8_t *e) {
  uint64_t k = 0;
  for (int v = 0; v < PL_MAXV; ++v) k |= (uint64_t)(e[v] & 7) << (3 * v);
  return k;
}

static int mdeg(const uint8_t *e) {
  int s = 0;
  for (int v = 0; v < PL_MAXV; ++v) s += e[v];
  return s;
}

/* ---------------------------------------------------------------- representative table */

typedef struct { uint64_t key; int64_t sidx; int32_t i, j; } occ_t;

static int occ_cmp(const void *a, const void *b) {
  const occ_t *x = (const occ_t *)a, *y = (const occ_t *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->sidx != y->sidx) return x->sidx < y->sidx ? -1 : 1;
  return 0;
}

typedef struct { int n; occ_t *r; } rep_table;

/* For every monomial of M = l([z]_2 [z]_2^T): the upper entry that comes first in svec order. */
static void build_reps(int nM, const mono_t *B2, rep_table *T) {
  int64_t ntri = (int64_t)nM * (nM + 1) / 2;
  occ_t *all = (occ_t *)malloc(sizeof(occ_t) * (size_t)ntri);
  int64_t q = 0;
  for (int j = 0; j < nM; ++j)
    for (int i = 0; i <= j; ++i) {
      uint8_t e[PL_MAXV];
      for (int v = 0; v < PL_MAXV; ++v) e[v] = (uint8_t)(B2[i][v] + B2[j][v]);
      all[q].key = mkey(e);
      all[q].sidx = (int64_t)j * (j + 1) / 2 + i;
      all[q].i = i;
      all[q].j = j;
      q++;
    }
  qsort(all, (size_t)ntri, sizeof(occ_t), occ_cmp);
  T->r = (occ_t *)malloc(sizeof(occ_t) * (size_t)ntri);
  T->n = 0;
  for (int64_t p = 0; p < ntri; ++p)
    if (p == 0 || all[p].key != all[p - 1].key) T->r[T->n++] = all[p];
  free(all);
}

static const occ_t *find_rep(const rep_table *T, const uint8_t *e) {
  uint64_t k = mkey(e);
  int lo = 0, hi = T->n - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (T->r[mid].key == k) return &T->r[mid];
    if (T->r[mid].key < k) lo = mid + 1; else hi = mid - 1;
  }
  return NULL;
}

/* ---------------------------------------------------------------- CSR row assembly */

typedef struct {
  int64_t nnz, cap;
  int32_t *col;
  double *val;
  int32_t m, mcap;
  int64_t *rowptr;
  double *b;
  int32_t *kind, *clique;
} rowbuf;

static void rb_add(rowbuf *R, int64_t col, double v) {
  if (R->nnz == R->cap) {
    R->cap = R->cap ? 2 * R->cap : 1024;
    R->col = (int32_t *)realloc(R->col, sizeof(int32_t) * (size_t)R->cap);
    R->val = (double *)realloc(R->val, sizeof(double) * (size_t)R->cap);
  }
  R->col[R->nnz] = (int32_t)col;
  R->val[R->nnz] = v;
  R->nnz++;
}

/* Coefficient `coef` on the matrix entry (i, j) of the block at svec offset `off`,
 * expressed on the svec coordinate (the sqrt(2) of svec is undone for off-diagonals). */
static void rb_entry(rowbuf *R, int64_t off, int i, int j, double coef) {
  if (i > j) { int t = i; i = j; j = t; }
  int64_t s = off + (int64_t)j * (j + 1) / 2 + i;
  rb_add(R, s, i == j ? coef : coef * M_SQRT1_2);
}

/* Close the current row: sort by column, merge duplicates, drop zeros. */
static void rb_end(rowbuf *R, int kind, int clique, double bval) {
  if (R->m + 1 >= R->mcap) {
    R->mcap = R->mcap ? 2 * R->mcap : 1024;
    R->rowptr = (int64_t *)realloc(R->rowptr, sizeof(int64_t) * (size_t)(R->mcap + 1));
    R->b = (double *)realloc(R->b, sizeof(double) * (size_t)R->mcap);
    R->kind = (int32_t *)realloc(R->kind, sizeof(int32_t) * (size_t)R->mcap);
    R->clique = (int32_t *)realloc(R->clique, sizeof(int32_t) * (size_t)R->mcap);
  }
  int64_t s = R->m == 0 ? 0 : R->rowptr[R->m];
  if (R->m == 0) R->rowptr[0] = 0;
  /* insertion sort: rows are short */
  for (int64_t p = s + 1; p < R->nnz; ++p) {
    int32_t c = R->col[p];
    double v = R->val[p];
    int64_t q = p - 1;
    while (q >= s && R->col[q] > c) {
      R->col[q + 1] = R->col[q];
      R->val[q + 1] = R->val[q];
      q--;
    }
    R->col[q + 1] = c;
    R->val[q + 1] = v;
  }
  int64_t w = s;
  for (int64_t p = s; p < R->nnz; ++p) {
    if (w > s && R->col[w - 1] == R->col[p]) R->val[w - 1] += R->val[p];
    else { R->col[w] = R->col[p]; R->val[w] = R->val[p]; w++; }
  }
  int64_t w2 = s;
  for (int64_t p = s; p < w; ++p)
    if (R->val[p] != 0.0) { R->col[w2] = R->col[p]; R->val[w2] = R->val[p]; w2++; }
  R->nnz = w2;
  R->b[R->m] = bval;
  R->kind[R->m] = kind;
  R->clique[R->m] = clique;
  R->m++;
  R->rowptr[R->m] = R->nnz;
}

static int64_t binom(int n, int k) {
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

/* ---------------------------------------------------------------- the relaxation */

int orc_relax(int family, int N, const double *prm, int nprm, orc_sdp **out) {
  int dx, du;
  double sx[PL_MAXV], su[PL_MAXV];
  *out = NULL;
  if (N < 1 || fam_layout(family, prm, nprm, &dx, &du, sx, su)) return -1;
  int lmap[PL_MAXV];
  const int dl = fam_lookahead(family, lmap);
  const int d = 2 * dx + du + dl;
  if (d > PL_MAXV) return -1;

  mono_t *B2 = NULL, *B1 = NULL;
  const int nM = basis(d, 2, &B2);
  const int n1 = basis(d, 1, &B1);
  if (nM != binom(d + 2, 2) || n1 != d + 1) return -2;
  rep_table T;
  build_reps(nM, B2, &T);

  pl_list *eq = (pl_list *)calloc((size_t)N, sizeof(pl_list));
  pl_list *iq = (pl_list *)calloc((size_t)N, sizeof(pl_list));
  pl_poly *cost = (pl_poly *)calloc((size_t)N, sizeof(pl_poly));
  int rc = 0;
  for (int k = 0; k < N && !rc; ++k) rc = fam_clique(family, N, k, prm, nprm, &eq[k], &iq[k], &cost[k]);

  /* degree checks of Prop. 1 with kappa = 2 */
  for (int k = 0; k < N && !rc; ++k) {
    for (int i = 0; i < eq[k].n; ++i) if (pl_deg(&eq[k].p[i]) > 4) rc = -3;
    for (int i = 0; i < iq[k].n; ++i) {
      int dg = pl_deg(&iq[k].p[i]);
      if (dg < 1 || dg > 2) rc = -3;
    }
    if (pl_deg(&cost[k]) > 4) rc = -3;
  }

  orc_sdp *P = (orc_sdp *)calloc(1, sizeof(orc_sdp));
  rowbuf R;
  memset(&R, 0, sizeof R);
  int64_t *offM = (int64_t *)calloc((size_t)N, sizeof(int64_t));
  int64_t **offL = (int64_t **)calloc((size_t)N, sizeof(int64_t *));

  if (!rc) {
    /* blocks: M_k followed by its localizing matrices */
    int nb = 0;
    for (int k = 0; k < N; ++k) nb += 1 + iq[k].n;
    P->nblocks = nb;
    P->bsize = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    P->bkind = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    P->bclique = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    P->boff = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
    int64_t off = 0;
    int bi = 0;
    for (int k = 0; k < N; ++k) {
      offM[k] = off;
      P->bsize[bi] = nM; P->bkind[bi] = 0; P->bclique[bi] = k; P->boff[bi] = off;
      off += (int64_t)nM * (nM + 1) / 2;
      bi++;
      offL[k] = (int64_t *)calloc((size_t)(iq[k].n + 1), sizeof(int64_t));
      for (int i = 0; i < iq[k].n; ++i) {
        offL[k][i] = off;
        int nL = n1; /* every inequality has degree 1 or 2, so its basis is [z]_1 */
        P->bsize[bi] = nL; P->bkind[bi] = 1; P->bclique[bi] = k; P->boff[bi] = off;
        off += (int64_t)nL * (nL + 1) / 2;
        bi++;
      }
    }
    P->nsvec = off;

    /* normalization phi_0 = 1: M_0(1,1) = 1 */
    rb_entry(&R, offM[0], 0, 0, 1.0);
    rb_end(&R, ORC_ROW_NORM, 0, 1.0);

    for (int k = 0; k < N; ++k) {
      /* (1) moment rows: every non-representative upper entry equals its representative */
      for (int j = 0; j < nM; ++j)
        for (int i = 0; i <= j; ++i) {
          uint8_t e[PL_MAXV];
          for (int v = 0; v < PL_MAXV; ++v) e[v] = (uint8_t)(B2[i][v] + B2[j][v]);
          const occ_t *r = find_rep(&T, e);
          if (r->i == i && r->j == j) continue;
          rb_entry(&R, offM[k], i, j, 1.0);
          rb_entry(&R, offM[k], r->i, r->j, -1.0);
          rb_end(&R, ORC_ROW_MOMENT, k, 0.0);
        }
      /* (2) localizing rows: L(a,b) - sum_t g_t M(rep(beta_a + beta_b + t)) = 0 */
      for (int gi = 0; gi < iq[k].n; ++gi) {
        const pl_poly *g = &iq[k].p[gi];
        for (int bb = 0; bb < n1; ++bb)
          for (int a = 0; a <= bb; ++a) {
            rb_entry(&R, offL[k][gi], a, bb, 1.0);
            for (int t = 0; t < g->n; ++t) {
              uint8_t e[PL_MAXV];
              for (int v = 0; v < PL_MAXV; ++v) e[v] = (uint8_t)(B1[a][v] + B1[bb][v] + g->t[t].e[v]);
              const occ_t *r = find_rep(&T, e);
              rb_entry(&R, offM[k], r->i, r->j, -g->t[t].c);
            }
            rb_end(&R, ORC_ROW_LOCALIZING, k, 0.0);
          }
      }
      /* (3) equality rows: l(h * m) = 0 for every m in [z]_{4 - deg h}, in basis order */
      for (int hi = 0; hi < eq[k].n; ++hi) {
        const pl_poly *h = &eq[k].p[hi];
        mono_t *Bm = NULL;
        const int nm = basis(d, 4 - pl_deg(h), &Bm);
        for (int q = 0; q < nm; ++q) {
          for (int t = 0; t < h->n; ++t) {
            uint8_t e[PL_MAXV];
            for (int v = 0; v < PL_MAXV; ++v) e[v] = (uint8_t)(Bm[q][v] + h->t[t].e[v]);
            const occ_t *r = find_rep(&T, e);
            rb_entry(&R, offM[k], r->i, r->j, h->t[t].c);
          }
          rb_end(&R, ORC_ROW_EQUALITY, k, 0.0);
        }
        free(Bm);
      }
      /* (4) consensus rows with clique k+1: every monomial of degree <= 4 in the variables the
       * two cliques share, x_{k+1} and the lookahead components of x_{k+2} (in that order) */
      if (k + 1 < N) {
        mono_t *Bx = NULL;
        const int nx = basis(dx + dl, 4, &Bx);
        for (int q = 0; q < nx; ++q) {
          uint8_t ek[PL_MAXV], ek1[PL_MAXV];
          memset(ek, 0, sizeof ek);
          memset(ek1, 0, sizeof ek1);
          for (int v = 0; v < dx; ++v) {
            ek[dx + du + v] = Bx[q][v]; /* x_{k+1} follows u_k in clique k */
            ek1[v] = Bx[q][v];          /* and is first in clique k+1      */
          }
          for (int j = 0; j < dl; ++j) {
            ek[2 * dx + du + j] = Bx[q][dx + j];         /* lookahead of clique k          */
            ek1[dx + du + lmap[j]] = Bx[q][dx + j];      /* part of x_{k+2} in clique k+1  */
          }
          const occ_t *r0 = find_rep(&T, ek), *r1 = find_rep(&T, ek1);
          rb_entry(&R, offM[k], r0->i, r0->j, 1.0);
          rb_entry(&R, offM[k + 1], r1->i, r1->j, -1.0);
          rb_end(&R, ORC_ROW_CONSENSUS, k, 0.0);
        }
        free(Bx);
      }
    }

    /* objective: <C_k, M_k> = sum_alpha c_alpha phi_alpha with c_alpha on the representative */
    P->C = (double *)calloc((size_t)P->nsvec, sizeof(double));
    for (int k = 0; k < N; ++k)
      for (int t = 0; t < cost[k].n; ++t) {
        const occ_t *r = find_rep(&T, cost[k].t[t].e);
        int64_t s = offM[k] + (int64_t)r->j * (r->j + 1) / 2 + r->i;
        P->C[s] += r->i == r->j ? cost[k].t[t].c : cost[k].t[t].c * M_SQRT1_2;
      }

    P->m = R.m;
    P->nnz = R.nnz;
    P->rowptr = R.rowptr;
    P->col = R.col;
    P->val = R.val;
    P->b = R.b;
    P->rowkind = R.kind;
    P->rowclique = R.clique;
    P->nclique_vars = d;
    P->dx = dx;
    P->du = du;
  }

  for (int k = 0; k < N; ++k) {
    pl_list_free(&eq[k]);
    pl_list_free(&iq[k]);
    pl_free(&cost[k]);
    free(offL[k]);
  }
  free(eq); free(iq); free(cost); free(offM); free(offL);
  free(B2); free(B1); free(T.r);
  if (rc) { orc_sdp_free(P); return rc; }
  *out = P;
  return 0;
}

void orc_sdp_free(orc_sdp *p) {
  if (!p) return;
  free(p->bsize); free(p->bkind); free(p->bclique); free(p->boff);
  free(p->rowptr); free(p->col); free(p->val); free(p->b); free(p->C);
  free(p->rowkind); free(p->rowclique);
  free(p);
}

/* ---------------------------------------------------------------- rank-one lifting */

static double mono_eval(const uint8_t *e, const double *z) {
  double t = 1.0;
  for (int v = 0; v < PL_MAXV; ++v)
    for (int k = 0; k < e[v]; ++k) t *= z[v];
  return t;
}

/* X(z) of the refined-certificate subsection: M_k(z) = [z]_2 [z]_2^T and
 * L_{k,i}(z) = g_{k,i}(z) [z]_1 [z]_1^T, in svec form; returns sum_k f_k(z). */
double orc_lift(int family, int N, const double *prm, int nprm, const double *z, double *X) {
  int dx, du;
  double sx[PL_MAXV], su[PL_MAXV];
  if (N < 1 || fam_layout(family, prm, nprm, &dx, &du, sx, su)) return NAN;
  int lmap[PL_MAXV];
  const int dl = fam_lookahead(family, lmap);
  const int d = 2 * dx + du + dl;
  mono_t *B2 = NULL, *B1 = NULL;
  const int nM = basis(d, 2, &B2);
  const int n1 = basis(d, 1, &B1);
  double obj = 0.0;
  int64_t off = 0;
  double *v = (double *)malloc(sizeof(double) * (size_t)nM);
  for (int k = 0; k < N; ++k) {
    double zc[PL_MAXV];
    memset(zc, 0, sizeof zc);
    for (int i = 0; i < 2 * dx + du; ++i) zc[i] = z[(int64_t)k * (dx + du) + i];
    for (int j = 0; j < dl; ++j) /* x_{k+2}, or past x_N the trailing lookahead values */
      zc[2 * dx + du + j] = k + 2 <= N ? z[(int64_t)(k + 2) * (dx + du) + lmap[j]]
                                       : z[(int64_t)N * (dx + du) + dx + j];
    pl_list eq = {0, 0, NULL}, iq = {0, 0, NULL};
    pl_poly cost;
    fam_clique(family, N, k, prm, nprm, &eq, &iq, &cost);
    obj += pl_eval(&cost, zc);
    for (int i = 0; i < nM; ++i) v[i] = mono_eval(B2[i], zc);
    for (int j = 0; j < nM; ++j)
      for (int i = 0; i <= j; ++i) {
        if (X) X[off] = (i == j ? 1.0 : M_SQRT2) * v[i] * v[j];
        off++;
      }
    for (int gi = 0; gi < iq.n; ++gi) {
      double gv = pl_eval(&iq.p[gi], zc);
      for (int j = 0; j < n1; ++j)
        for (int i = 0; i <= j; ++i) {
          if (X) X[off] = (i == j ? 1.0 : M_SQRT2) * gv * v[i] * v[j]; /* [z]_1 is a prefix of [z]_2 */
          off++;
        }
    }
    pl_list_free(&eq);
    pl_list_free(&iq);
    pl_free(&cost);
  }
  free(v); free(B2); free(B1);
  return obj;
}

double orc_rollout(int family, int N, const double *prm, int nprm, const double *u, double *z) {
  int dx, du;
  double sx[PL_MAXV], su[PL_MAXV];
  if (N < 1 || fam_layout(family, prm, nprm, &dx, &du, sx, su)) return NAN;
  double x[PL_MAXV], x1[PL_MAXV], uk[PL_MAXV], aux[PL_MAXV];
  int lmap[PL_MAXV];
  const int dl = fam_lookahead(family, lmap);
  if (fam_init_state(family, prm, nprm, x) || fam_init_aux(family, prm, nprm, aux)) return NAN;
  for (int k = 0; k < N; ++k) {
    for (int i = 0; i < du; ++i) uk[i] = u[(int64_t)k * du + i];
    if (fam_step(family, prm, nprm, x, uk, x1, aux)) return NAN;
    for (int i = 0; i < dx; ++i) z[(int64_t)k * (dx + du) + i] = x[i];
    for (int i = 0; i < du; ++i) z[(int64_t)k * (dx + du) + dx + i] = uk[i];
    memcpy(x, x1, sizeof x);
  }
  for (int i = 0; i < dx; ++i) z[(int64_t)N * (dx + du) + i] = x[i];
  if (dl > 0) {
    /* the lookahead components of x_{N+1} (those of the families here do not depend on the
     * control of that step) */
    for (int i = 0; i < du; ++i) uk[i] = 0;
    if (fam_step(family, prm, nprm, x, uk, x1, aux)) return NAN;
    for (int j = 0; j < dl; ++j) z[(int64_t)N * (dx + du) + dx + j] = x1[lmap[j]];
  }
  return orc_lift(family, N, prm, nprm, z, NULL);
}

/* Trace bounds for the certificate (App. "Existence of R_beta", with the square that the proof
 * drops restored): if every variable of clique k satisfies |z_v| <= R_k, each monomial of
 * degree t of the basis is at most max(1, R_k)^t in size, so for the rank-one lifting
 *   tr M_k(z) = ||[z]_2||^2 <= s(d, 2) * max(1, R_k)^4,
 *   tr L_{k,i}(z) = g(z) ||[z]_1||^2 <= (max of g over the box |z| <= R_k) * s(d, 1) * max(1, R_k)^2.
 * The maximum of g is bounded term by term: exactly for the one-variable terms of degree <= 2
 * of each variable together, by |c| R^deg for every other term (the car back-in's separation
 * inequalities are products of two variables).  R_beta: nblocks values. */
static int dbl_cmp(const void *x, const void *y) {
  const double u = *(const double *)x, v = *(const double *)y;
  return u < v ? -1 : (u > v ? 1 : 0);
}

static int box_max_sep(const pl_poly *g, double R, double *out) {
  double a[PL_MAXV] = {0}, b[PL_MAXV] = {0}, c = 0;
  double *mixed = (double *)malloc(sizeof(double) * (size_t)(g->n + 1));
  int nmixed = 0;
  for (int t = 0; t < g->n; ++t) {
    int var = -1, e = 0, deg = 0, nv = 0;
    for (int v = 0; v < PL_MAXV; ++v)
      if (g->t[t].e[v]) {
        var = v;
        e = g->t[t].e[v];
        deg += e;
        nv++;
      }
    if (nv == 0) c += g->t[t].c;
    else if (nv == 1 && e == 2) a[var] += g->t[t].c;
    else if (nv == 1 && e == 1) b[var] += g->t[t].c;
    else {  /* any other term: at most |c| R^deg on the box */
      double m = fabs(g->t[t].c);
      for (int q = 0; q < deg; ++q) m *= R;
      mixed[nmixed++] = m;
    }
  }
  for (int v = 0; v < PL_MAXV; ++v) {
    if (a[v] == 0 && b[v] == 0) continue;
    double best = fmax(a[v] * R * R + b[v] * R, a[v] * R * R - b[v] * R);
    if (a[v] != 0) {
      const double t = -b[v] / (2 * a[v]);
      if (fabs(t) <= R) best = fmax(best, a[v] * t * t + b[v] * t);
    }
    c += best;
  }
  /* the bounds of the other terms, summed in ascending order */
  qsort(mixed, (size_t)nmixed, sizeof(double), dbl_cmp);
  double sm = 0;
  for (int q = 0; q < nmixed; ++q) sm += mixed[q];
  free(mixed);
  *out = c + sm;
  return 0;
}

int orc_trace_bounds(int family, int N, const double *prm, int nprm, double *R_beta) {
  int dx, du;
  double sx[PL_MAXV], su[PL_MAXV], bnd[PL_MAXV];
  if (N < 1 || fam_layout(family, prm, nprm, &dx, &du, sx, su)) return -1;
  if (fam_var_bounds(family, prm, nprm, bnd)) return -2;
  int lmap[PL_MAXV];
  const int dl = fam_lookahead(family, lmap);
  for (int j = 0; j < dl; ++j) bnd[2 * dx + du + j] = bnd[lmap[j]];
  const int d = 2 * dx + du + dl;
  double R0 = 0;
  for (int v = 0; v < d; ++v) R0 = fmax(R0, bnd[v]);
  const double sM = (double)binom(d + 2, 2), s1 = (double)(d + 1);
  int bi = 0, rc = 0;
  for (int k = 0; k < N && !rc; ++k) {
    /* R_k: the last clique also holds the lookahead past the horizon */
    const double Rk = k == N - 1 ? fmax(R0, fam_tail_bound(family, prm, nprm)) : R0;
    const double r1 = fmax(1.0, Rk);
    pl_list eq, iq;
    pl_poly cost;
    memset(&eq, 0, sizeof eq);
    memset(&iq, 0, sizeof iq);
    rc = fam_clique(family, N, k, prm, nprm, &eq, &iq, &cost);
    if (!rc) {
      R_beta[bi++] = sM * r1 * r1 * r1 * r1;
      for (int i = 0; i < iq.n && !rc; ++i) {
        double gm = 0;
        rc = box_max_sep(&iq.p[i], Rk, &gm);
        R_beta[bi++] = fmax(0.0, gm) * s1 * r1 * r1;
      }
    }
    pl_list_free(&eq);
    pl_list_free(&iq);
    pl_free(&cost);
  }
  return rc;
}
