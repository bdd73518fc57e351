/*
 * strom_gen.h -- C ABI of the host-side relaxation generator that feeds strom_sdp_setup.
 *
 * It builds the sparse second-order moment relaxation (relaxation order 2, Prop. 1 of
 * Kang et al., "Fast and Certifiable Trajectory Optimization", Sec. "Sparse Moment
 * Relaxation") of a polynomial trajectory-optimization problem with chain-like sparsity
 * (Def. 1) and converts it to the PSD-only multi-block standard SDP of the subsection
 * "Faster Conversion to Standard SDP": moment, localizing, equality and consensus rows plus
 * the normalization phi_0 = 1.  Output arrays follow strom.h (svec columns, CSR rows).
 * This is one-time setup on the host; nothing here runs in the ADMM iteration.
 *
 * Families (params are original-unit values, see each line):
 *   0 toy 1-D system of the paper's worked example   [x_init, dt, P_f]
 *   1 pendulum (7-variable cliques, 36x36 / 8x8)      [theta0, omega0]
 *   2 cart-pole (11-variable cliques, 78x78 / 12x12)  [x0, v0, theta0, omega0]
 *   3 the paper's variational-integrator pendulum     [theta0, omega0]
 *   4 planar car, unicycle-12 (91x91 / 13x13) or bicycle-13 (105x105 / 14x14)
 *                                                     [variant, sx, sy, heading0, gx, gy, ox, oy]
 *   5 the paper's flying robot (App. "Flying Robot"; 20-variable cliques, 231x231 / 21x21)
 *                                                     [x0, y0, theta0, vx0, vy0, omega0]
 *   6 the paper's vehicle landing (App. "Vehicle Landing"; 18-variable cliques, 190x190 / 19x19)
 *                                                     [x0, y0, theta0, vx0, vy0, omega0]
 *   7 the paper's car back-in (App. "Car Back-in"; 18-variable cliques, 190x190 / 19x19) [x0, y0, theta0]
 *   8 the paper's cart-pole (App. "Cart-Pole"; 13-variable cliques (x_k, u_k, x_{k+1}, a_{k+2},
 *     rs_{k+2}) that share 7 variables, 105x105 / 14x14)  [a0, adot0, theta0 from hanging, thetadot0]
 *
 * Every function returns 0 on success and a negative strom_status on error.
 */
#ifndef STROM_GEN_H
#define STROM_GEN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct strom_gen_sdp strom_gen_sdp;

/* Build the relaxation of one instance with horizon N (N >= 1).  E_INVAL (-1) on a bad
 * family, N or parameter count. */
int strom_gen_build(int family, int N, const double *params, int nparams, strom_gen_sdp **out);

/* Sizes of a built relaxation (any pointer may be NULL). */
int strom_gen_sizes(const strom_gen_sdp *g, int32_t *nblocks, int32_t *m, int64_t *nnz,
                    int64_t *n_svec);

/* Copy the relaxation out into caller-allocated host arrays: block_sizes[nblocks],
 * rowptr[m+1], col[nnz], val[nnz], b[m], C[n_svec]; row_kind[m] (nullable) receives
 * 0 normalization, 1 moment, 2 localizing, 3 equality, 4 consensus. */
int strom_gen_export(const strom_gen_sdp *g, int32_t *block_sizes, int64_t *rowptr, int32_t *col,
                     double *val, double *b, double *C_svec, int32_t *row_kind);

/* Trace bounds R_beta (nblocks values) of the certificate's valid lower bound (Sec.
 * "Algorithmic Backbone", the valid-lower-bound equation), from App. "Existence of R_beta": with
 * every scaled variable of clique k bounded by R_k (box constraints, unit circles and the
 * initial state of the family), R_beta = s(d, 2) max(1, R_k)^4 for M_k and
 * max_{|z| <= R_k} g_{k,i}(z) * s(d, 1) max(1, R_k)^2 for L_{k,i}, the maximum taken exactly for
 * the one-variable terms of degree <= 2 and as |c| R_k^deg for every other term.  (The cart-pole
 * of the paper bounds its last clique's lookahead a_{N+1} through the dynamics.)  (The appendix
 * writes s(d, 2) R_k^2,
 * which is not a bound when R_k < 1 or for the degree-two monomials; max(1, R_k)^(2 deg) bounds
 * the square of every monomial of the basis.)  E_INVAL when a variable of the family has no
 * bound (the pendulum's angular rate). */
int strom_gen_trace_bounds(const strom_gen_sdp *g, double *R_beta);

void strom_gen_free(strom_gen_sdp *g);

#ifdef __cplusplus
}
#endif
#endif
