// Internal declarations shared by the host table builder and the HIP library.
#ifndef SEDG_INTERNAL_H
#define SEDG_INTERNAL_H

#define MAXN 8

// Operator tables of one DG level n; matrices are row-major with row stride n.
struct sedg_level_tab {
    int n;
    int pad;
    double xi[MAXN], w[MAXN];
    double Dcal[MAXN * MAXN];   // l_j'(xi_i)
    double D[MAXN * MAXN];      // M^-1 Dcal^T M
    double bm[MAXN], bp[MAXN];  // l_j(-1/2), l_j(+1/2)
    double P[MAXN * MAXN];      // projection nodal -> subcell means
    double R[MAXN * MAXN];      // reconstruction subcell means -> nodal
    double Dhat[MAXN * MAXN];   // P D
    double Bhl[MAXN], Bhr[MAXN];// nonzero columns of P B^(0)
    double Ip[MAXN * MAXN];     // l_j(mu_{i+1/2})
    double Im[MAXN * MAXN];     // l_j(mu_{i-1/2})
    double Ep[MAXN * MAXN];     // Ip R
    double Em[MAXN * MAXN];     // Im R
    // transposes, for the adjoint
    double RT[MAXN * MAXN], PT[MAXN * MAXN], DhatT[MAXN * MAXN], EpT[MAXN * MAXN], EmT[MAXN * MAXN];
};

int sedg_build_level(int n, int family, sedg_level_tab *T);

// Tables of the refinement / coarsening and mortar operators of level n (App.,
// non-conforming interfaces); matrices row-major.
struct sedg_nc_tab {
    int n;
    int pad;
    double Z[2 * MAXN * MAXN];   // P^(n -> 2n): n nodal values -> 2n subcell means (2n x n)
    double Q[MAXN * MAXN / 2];   // P^(n -> n/2): n nodal values -> n/2 subcell means (n/2 x n)
    double Lm[MAXN * MAXN];      // L_-: l_i(xi_j / 2 - 1/4) w_j / (2 w_i)  (n x n)
    double Lp[MAXN * MAXN];      // L_+: l_i(xi_j / 2 + 1/4) w_j / (2 w_i)  (n x n)
};

int sedg_build_nc(int n, int family, sedg_nc_tab *T);

#endif
