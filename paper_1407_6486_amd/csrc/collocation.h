// Host-side construction of the collocation matrices (Sec. 2.1, eq. Qbe).
#pragma once

namespace pfmg {

// Gauss-Lobatto nodes on [0, 1] in long double; false if nnodes outside 2..16.
bool lobatto_nodes_ld(int nnodes, long double *s);
// Nodes of a family (PFMG_NODES_LOBATTO, PFMG_NODES_UNIFORM: m / M).
bool family_nodes_ld(int family, int nnodes, long double *s);
// Q (nn x nn), S ((nn-1) x nn), d (nn) rounded once to double.  first = 0:
// the quadrature interpolates f through every node; first = 1: through
// nodes 1..M only (column 0 of Q is zero).
bool collocation_matrices(int nnodes, const long double *s, double *Q, double *S, double *d, int first = 0);
// L[mf][mc] = l^c_mc(sf[mf]).
void lagrange_interp(int nf, const long double *sf, int nc, const long double *sc, double *L);

}  // namespace pfmg
