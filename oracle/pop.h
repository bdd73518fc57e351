/* pop.h -- oracle-internal polynomial type and family builders (TEST INFRASTRUCTURE ONLY). */
#ifndef STROM_ORACLE_POP_H
#define STROM_ORACLE_POP_H
#include <stdint.h>

#include "oracle.h"

#define PL_MAXV 21 /* max variables per clique (3-bit exponents of 21 variables fit a 64-bit key) */

typedef struct { uint8_t e[PL_MAXV]; double c; } pl_term;
typedef struct { int n, cap; pl_term *t; } pl_poly;
typedef struct { int n, cap; pl_poly *p; } pl_list;

void pl_init(pl_poly *p);
void pl_free(pl_poly *p);
void pl_combine(pl_poly *p);
pl_poly pl_copy(const pl_poly *a);
pl_poly pl_const(double c);
pl_poly pl_var(int i, double c);
pl_poly pl_axpy(const pl_poly *a, double s, const pl_poly *b);
pl_poly pl_mul(const pl_poly *a, const pl_poly *b);
int pl_deg(const pl_poly *p);
void pl_normalize(pl_poly *p);
double pl_eval(const pl_poly *p, const double *z);
void pl_list_free(pl_list *l);

int fam_layout(int family, const double *prm, int nprm, int *dx, int *du, double *sx, double *su);
int fam_clique(int family, int N, int k, const double *prm, int nprm, pl_list *eq, pl_list *ineq,
               pl_poly *cost);
int fam_lookahead(int family, int *lmap);
int fam_step(int family, const double *prm, int nprm, const double *x0, double *u, double *x1, double *aux);
int fam_init_state(int family, const double *prm, int nprm, double *x0);
int fam_init_aux(int family, const double *prm, int nprm, double *aux);
int fam_var_bounds(int family, const double *prm, int nprm, double *bnd);
double fam_tail_bound(int family, const double *prm, int nprm);

#endif
