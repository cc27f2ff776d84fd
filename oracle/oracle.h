/*
 * Plain FP64 CPU oracle for IPFASST interwoven with geometric multigrid
 * (Minion, Speck, Bolten, Emmett, Ruprecht, "Interweaving PFASST and
 * Parallel Multigrid", arXiv:1407.6486).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant generator with the HIP library; the two
 * sides meet only through seeded inputs.
 *
 * Grids are dense arrays of n^dim interior values (no halo), x fastest:
 * index(i,j,k) = i + n*(j + n*k), 0-based.  Homogeneous Dirichlet data
 * lives outside the array: a neighbour outside [0,n) reads as zero.
 * Mesh width h = 1/(n+1) (interior points x_i = (i+1) h).
 *
 * Every routine follows the algorithm in the order the paper states it;
 * nothing is blocked, fused or reordered.  Where the paper is silent the
 * reading used is stated at the routine.
 */
#ifndef PFASST_ORACLE_H
#define PFASST_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- nodes */
/* Gauss-Lobatto nodes on [0,1] (nnodes = M+1 >= 2), long double Newton on
 * the derivative of the Legendre polynomial, rounded once to double. */
int or_lobatto_nodes(int nnodes, double *s);

/* Node families: Gauss-Lobatto (the quadrature uses every node), and the
 * paper's uniform nodes s_m = m/M whose quadrature leaves out the left end
 * point (Sec. 3: q_{m,0} = 0, the interpolant of f runs through nodes
 * 1..M; M = 1 is backward Euler, M = 2 the second-order and M = 4 the
 * fourth-order method of the 3D runs in Sec. 4). */
enum { OR_NODES_LOBATTO = 0, OR_NODES_UNIFORM = 1 };
/* s_m = m / (nnodes - 1), exactly. */
int or_uniform_nodes(int nnodes, double *s);
/* As or_qmat for either family: family OR_NODES_UNIFORM builds every row
 * from the Lagrange basis of the nodes s_1..s_M (column 0 stays zero). */
int or_qmat_family(int nnodes, const double *s, int family, double *Q, double *S, double *d);

/* Integration matrix Q[m][i] = int_0^{s_m} l_i(s) ds (Sec. 2.1; first row
 * zero), the node-to-node matrix S[m][i] = Q[m+1][i]-Q[m][i] (eq. sdc-be,
 * (M)x(M+1)), and the backward-Euler substeps d[m] = s_m - s_{m-1}
 * (eq. Qbe, d[0]=0).  All computed in long double, rounded once. */
int or_qmat(int nnodes, const double *s, double *Q, double *S, double *d);

/* Lagrange interpolation matrix from coarse nodes sc (ncn) to fine nodes
 * sf (nfn): L[mf][mc] = l^c_mc(sf[mf]). */
int or_interp_matrix(int nfn, const double *sf, int ncn, const double *sc,
                     double *L);

/* ------------------------------------------------------------ stencils */
/* out = L_h u, the 2nd-order (2*dim+1)-point Laplacian, Dirichlet 0. */
void or_lap(int dim, int n, const double *u, double *out);
/* out = (I - alpha L_h) u. */
void or_helm(int dim, int n, double alpha, const double *u, double *out);
/* r = b - (I - alpha L_h) u. */
void or_resid(int dim, int n, double alpha, const double *b, const double *u,
              double *r);
double or_norm_inf(size_t len, const double *v);

/* -------------------------------------------------------- multigrid
 * smoother: 0 = weighted Jacobi (weight omega), 1 = red-black Gauss-Seidel
 * (red = (i+j+k) even in 1-based interior indices, red then black, relaxed
 * with weight omega; omega = 1 is plain Gauss-Seidel). */
enum { OR_JACOBI = 0, OR_RBGS = 1 };

void or_smooth(int dim, int n, double alpha, int smoother, double omega,
               const double *b, double *u);
/* Full weighting (1/4,1/2,1/4)^dim of a fine array onto the coarse grid
 * nc = (n+1)/2 - 1. */
void or_restrict_fw(int dim, int n, const double *r, double *bc);
/* u += P ec, d-linear interpolation with zero boundary values. */
void or_prolong_add(int dim, int nc, const double *ec, double *u);
/* u += P4 ec: tensor-product cubic (fourth-order) Lagrange interpolation.
 * A fine point on a coarse point takes that value; a fine point between
 * coarse points J and J+1 interpolates the cubic through J-1..J+2, shifted
 * inwards next to the boundary (the boundary value 0 is one of the four
 * points).  Needs nc >= 3. */
void or_prolong4_add(int dim, int nc, const double *ec, double *u);
/* Fourth-order discretisation (Sec. 4.3): L4 with odd reflection beyond
 * the boundary, its residual, smoother (weighted Jacobi or red-black JOR,
 * each colour from the values before its pass), a V-cycle whose finest
 * level uses L4 above the second-order V-cycle, and the solve policy. */
void or_lap4(int dim, int n, const double *u, double *out);
void or_resid4(int dim, int n, double alpha, const double *b, const double *u, double *r);
void or_smooth4(int dim, int n, double alpha, int smoother, double omega, const double *b, double *u);
void or_vcycle4(int dim, int n, double alpha, int smoother, double omega, int nu1, int nu2,
                const double *b, double *u);
/* Exact solve of (I - alpha L_h) u = b for n in {1,2}. */
void or_coarsest(int dim, int n, double alpha, const double *b, double *u);
/* One V(nu1,nu2)-cycle on (I - alpha L_h) u = b, in place on u. */
void or_vcycle(int dim, int n, double alpha, int smoother, double omega,
               int nu1, int nu2, const double *b, double *u);

/* Single-precision twins of the multigrid routines (used by the mixed
 * precision form: FP32 smoothing, restriction, prolongation inside FP64
 * iterative refinement).  Coefficients are formed in double and rounded
 * once to float. */
void orf_smooth(int dim, int n, double alpha, int smoother, double omega,
                const float *b, float *u);
void orf_resid(int dim, int n, double alpha, const float *b, const float *u,
               float *r);
void orf_restrict_fw(int dim, int n, const float *r, float *bc);
void orf_prolong_add(int dim, int nc, const float *ec, float *u);
void orf_coarsest(int dim, int n, double alpha, const float *b, float *u);
void orf_vcycle(int dim, int n, double alpha, int smoother, double omega,
                int nu1, int nu2, const float *b, float *u);

/* Solve policy for one implicit node solve. */
typedef struct or_mg_policy {
    int smoother;     /* OR_JACOBI / OR_RBGS */
    int nu1, nu2;     /* pre / post smoothing sweeps */
    double omega;     /* smoother weight */
    int cycles;       /* > 0: exactly this many V-cycles; 0: to tolerance */
    double tol;       /* stop when |b - H u|_inf <= tol |b|_inf (cycles==0) */
    double stall;     /* stop when |r_new| >= stall |r_old| (cycles==0) */
    int max_cycles;   /* cap (cycles==0) */
    int mixed;        /* 1: FP32 V-cycle inside FP64 iterative refinement */
} or_mg_policy;

/* Returns the number of V-cycles run; *relres = |b - H u|_inf / |b|_inf
 * after the last cycle (computed only when relres != NULL). */
int or_mg_solve(int dim, int n, double alpha, const or_mg_policy *pol,
                const double *b, double *u, double *relres);
/* The same for (I - alpha L4) (FP64 only). */
int or_mg_solve4(int dim, int n, double alpha, const or_mg_policy *pol,
                 const double *b, double *u, double *relres);

/* ---------------------------------------------------------------- PFASST */
typedef struct or_params {
    int dim, n;              /* fine grid */
    double nu, dt;           /* diffusion coefficient, slice length */
    int n_slices;            /* P */
    int nodes_fine;          /* M_f + 1 */
    int nodes_coarse;        /* M_c + 1, 0 = single level (ISDC) */
    or_mg_policy mg;         /* policy for every node solve (both levels) */
    int interp_order;        /* PFASST spatial interpolation: 2 d-linear, 4 cubic */
    int node_family;         /* OR_NODES_LOBATTO / OR_NODES_UNIFORM */
    int stencil_order;       /* fine-level Laplacian: 2, or 4 (coarse level stays 2) */
    int f_solve;             /* F at a node after its solve: 0 nu L U; 1 (U - b) / (dt d_m),
                              * the value the implicit-Euler substep implies (both levels) */
    int f_interp;            /* after the coarse correction: 0 F_f re-evaluated; 1 the
                              * coarse F correction interpolated like U's */
    int residual_abs;        /* collocation residual: 0 relative to |U0_p|_inf, 1 absolute */
    int nodes_middle;        /* > 0: three levels, this many nodes on the middle one
                              * (needs nodes_coarse > 0) */
    int fine_send;           /* new fine initial value of slice p at iteration k+1: 0 slice
                              * p-1's end value after iteration k (after the coarse
                              * correction); 1 its end value right after its fine sweep of
                              * iteration k (Sec. 2.4, sent after the sweep) */
} or_params;

typedef struct or_pfasst or_pfasst;

or_pfasst *or_pfasst_create(const or_params *prm);
void or_pfasst_destroy(or_pfasst *c);
/* Spread u_block to every node of every slice (and the FAS restriction /
 * predictor when two levels are present). */
void or_pfasst_spread(or_pfasst *c, const double *u_block);
void or_pfasst_predictor(or_pfasst *c);
/* One IPFASST iteration; returns the block residual. */
double or_pfasst_iter(or_pfasst *c);
/* Block residual (eq. resid), per slice into res[P] (may be NULL). */
double or_pfasst_residual(or_pfasst *c, double *res);
/* One SDC sweep on slice p at level 0 (fine) or 1 (coarse, with tau). */
void or_sdc_sweep(or_pfasst *c, int level, int p);
/* FAS restriction of slice p and interpolation of slice p (levels 0 and
 * 1), and the same between levels l and l+1. */
void or_fas_restrict(or_pfasst *c, int p);
void or_interpolate(or_pfasst *c, int p);
void or_fas_restrict_level(or_pfasst *c, int l, int p);
void or_interpolate_level(or_pfasst *c, int l, int p);
/* Any level's field: kind 0 U, 1 F, 2 tau, 3 U^old (levels >= 1). */
enum { OR_K_U = 0, OR_K_F = 1, OR_K_TAU = 2, OR_K_UOLD = 3 };
double *or_pfasst_level_field(or_pfasst *c, int lev, int kind, int p, int m);

/* Field access.  which: 0 U_f, 1 F_f, 2 U_c, 3 F_c, 4 tau, 5 U_c_old,
 * 6 F_c_old (f_interp only). */
enum { OR_UF = 0, OR_FF = 1, OR_UC = 2, OR_FC = 3, OR_TAU = 4, OR_UCOLD = 5, OR_FCOLD = 6 };
double *or_pfasst_field(or_pfasst *c, int which, int p, int m);
/* Node solve counters (V-cycles run so far at each level). */
long long or_pfasst_vcycles(or_pfasst *c, int level);
void or_pfasst_matrices(or_pfasst *c, int level, double *s, double *Q);

#ifdef __cplusplus
}
#endif
#endif
