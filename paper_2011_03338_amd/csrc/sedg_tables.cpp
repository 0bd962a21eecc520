// Operator tables of the blended DG/FV scheme, built in quad precision on the
// host and rounded once to double.
//
// Per level n (the DG order of a sub-element, Sec. 2.2-2.4 and 2.6):
//   xi, w       collocation nodes on [-1/2, 1/2] and quadrature weights (sum 1):
//               Gauss-Legendre (the paper's choice) or Legendre-Gauss-Lobatto
//   Dcal        Dcal_ij = l_j'(xi_i), from barycentric weights
//   D           M^-1 Dcal^T M                        (eq. semi-discrete-dg)
//   bm, bp      l_j(-1/2), l_j(+1/2)                 (eq. boundary-interpolation-operators)
//   P           P_ij = n * mean of l_j over subcell i, by exact integration of the
//               monomial form of l_j                  (Sec. 2.3)
//   R           P^-1                                  (eq. trafo-mv-nodal)
//   Dhat, Bhat  P D and the two nonzero columns of P B^(0)  (eq. dgfv-operators)
//   Ip, Im      l_j(mu_{i+1/2}), l_j(mu_{i-1/2})       (eq. subcell-fv-interpolation-operator)
//   Ep, Em      Ip R, Im R: subcell means -> values at subcell interfaces
#include <quadmath.h>

#include <cstring>

#include "sedg_internal.h"

namespace {

typedef __float128 q;

// Legendre P_m(x) and P_m'(x) on [-1, 1].
void legendre(int m, q x, q &p, q &dp)
{
    q p0 = 1, p1 = x;
    if (m == 0) { p = 1; dp = 0; return; }
    for (int k = 2; k <= m; ++k) {
        q p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    // derivative from the recurrence m (P_{m-1} - x P_m) / (1 - x^2)
    dp = m * (p0 - x * p1) / (1 - x * x);
}

void gauss(int n, q *x, q *w)
{
    for (int i = 0; i < n; ++i) {
        // Tricomi's first guess for the i-th root (descending), refined by Newton
        q t = cosq(M_PIq * (4 * i + 3) / (4 * n + 2));
        for (int it = 0; it < 200; ++it) {
            q p, dp;
            legendre(n, t, p, dp);
            q d = p / dp;
            t -= d;
            if (fabsq(d) < 1e-33Q) break;
        }
        q p, dp;
        legendre(n, t, p, dp);
        x[n - 1 - i] = t / 2;
        w[n - 1 - i] = 1 / ((1 - t * t) * dp * dp);  // (2 / ((1-t^2) P'^2)) / 2
    }
}

void lobatto(int n, q *x, q *w)
{
    int N = n - 1;
    x[0] = -q(1) / 2;
    x[N] = q(1) / 2;
    for (int i = 1; i < N; ++i) {
        q t = -cosq(M_PIq * i / N);
        for (int it = 0; it < 200; ++it) {
            q p, dp;
            legendre(N, t, p, dp);
            // P_N'' from the Legendre equation
            q d2 = (2 * t * dp - N * (N + 1) * p) / (1 - t * t);
            q d = dp / d2;
            t -= d;
            if (fabsq(d) < 1e-33Q) break;
        }
        x[i] = t / 2;
    }
    for (int i = 0; i <= N; ++i) {
        q p, dp;
        legendre(N, 2 * x[i], p, dp);
        w[i] = 1 / (N * (N + 1) * p * p);
    }
}

// monomial coefficients c[0..n-1] of the Lagrange basis l_j
void lagrange_monomial(int n, const q *x, int j, q *c)
{
    q poly[MAXN + 1];
    for (int k = 0; k <= n; ++k) poly[k] = 0;
    poly[0] = 1;
    int deg = 0;
    q denom = 1;
    for (int k = 0; k < n; ++k) {
        if (k == j) continue;
        // multiply by (t - x_k)
        for (int d = deg + 1; d >= 1; --d) poly[d] = poly[d - 1] - x[k] * poly[d];
        poly[0] = -x[k] * poly[0];
        ++deg;
        denom *= (x[j] - x[k]);
    }
    for (int k = 0; k < n; ++k) c[k] = poly[k] / denom;
}

q polyval(int n, const q *c, q t)
{
    q s = 0;
    for (int k = n - 1; k >= 0; --k) s = s * t + c[k];
    return s;
}

// integral of the polynomial c over [a, b]
q polyint(int n, const q *c, q a, q b)
{
    q s = 0;
    for (int k = 0; k < n; ++k) s += c[k] * (powq(b, k + 1) - powq(a, k + 1)) / (k + 1);
    return s;
}

bool lu_inverse(int n, const q *A, q *Ainv)
{
    q a[MAXN][MAXN];
    int piv[MAXN];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) a[i][j] = A[i * n + j];
    for (int i = 0; i < n; ++i) piv[i] = i;
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabsq(a[i][k]) > fabsq(a[p][k])) p = i;
        if (a[p][k] == 0) return false;
        if (p != k) {
            for (int j = 0; j < n; ++j) { q t = a[k][j]; a[k][j] = a[p][j]; a[p][j] = t; }
            int t = piv[k]; piv[k] = piv[p]; piv[p] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            a[i][k] /= a[k][k];
            for (int j = k + 1; j < n; ++j) a[i][j] -= a[i][k] * a[k][j];
        }
    }
    // solve for each unit column
    for (int col = 0; col < n; ++col) {
        q y[MAXN];
        for (int i = 0; i < n; ++i) {
            q s = (piv[i] == col) ? 1 : 0;
            for (int j = 0; j < i; ++j) s -= a[i][j] * y[j];
            y[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            q s = y[i];
            for (int j = i + 1; j < n; ++j) s -= a[i][j] * y[j];
            y[i] = s / a[i][i];
        }
        for (int i = 0; i < n; ++i) Ainv[i * n + col] = y[i];
    }
    return true;
}

}  // namespace

int sedg_build_level(int n, int family, sedg_level_tab *T)
{
    if (n < 2 || n > MAXN || (n & (n - 1))) return -1;
    q x[MAXN], w[MAXN];
    if (family == 1) lobatto(n, x, w);
    else gauss(n, x, w);
    // barycentric weights
    q lam[MAXN];
    for (int j = 0; j < n; ++j) {
        q p = 1;
        for (int k = 0; k < n; ++k)
            if (k != j) p *= (x[j] - x[k]);
        lam[j] = 1 / p;
    }
    q Dc[MAXN * MAXN], Dv[MAXN * MAXN], P[MAXN * MAXN], R[MAXN * MAXN];
    for (int i = 0; i < n; ++i) {
        q diag = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            Dc[i * n + j] = (lam[j] / lam[i]) / (x[i] - x[j]);
            diag -= Dc[i * n + j];
        }
        Dc[i * n + i] = diag;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Dv[i * n + j] = Dc[j * n + i] * w[j] / w[i];
    q coef[MAXN][MAXN];
    for (int j = 0; j < n; ++j) lagrange_monomial(n, x, j, coef[j]);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            q a = -q(1) / 2 + q(i) / n, b = -q(1) / 2 + q(i + 1) / n;
            P[i * n + j] = n * polyint(n, coef[j], a, b);
        }
    if (!lu_inverse(n, P, R)) return -1;
    std::memset(T, 0, sizeof(*T));
    T->n = n;
    q bm[MAXN], bp[MAXN], Ip[MAXN * MAXN], Im[MAXN * MAXN];
    for (int j = 0; j < n; ++j) {
        bm[j] = polyval(n, coef[j], -q(1) / 2);
        bp[j] = polyval(n, coef[j], q(1) / 2);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            Ip[i * n + j] = polyval(n, coef[j], -q(1) / 2 + q(i + 1) / n);
            Im[i * n + j] = polyval(n, coef[j], -q(1) / 2 + q(i) / n);
        }
    for (int i = 0; i < n; ++i) {
        T->xi[i] = (double)x[i];
        T->w[i] = (double)w[i];
        T->bm[i] = (double)bm[i];
        T->bp[i] = (double)bp[i];
        q sl = 0, sr = 0;
        for (int k = 0; k < n; ++k) {
            sl += P[i * n + k] * (-bm[k] / w[k]);
            sr += P[i * n + k] * (bp[k] / w[k]);
        }
        T->Bhl[i] = (double)sl;
        T->Bhr[i] = (double)sr;
        for (int j = 0; j < n; ++j) {
            T->Dcal[i * n + j] = (double)Dc[i * n + j];
            T->D[i * n + j] = (double)Dv[i * n + j];
            T->P[i * n + j] = (double)P[i * n + j];
            T->R[i * n + j] = (double)R[i * n + j];
            T->Ip[i * n + j] = (double)Ip[i * n + j];
            T->Im[i * n + j] = (double)Im[i * n + j];
            q dh = 0, ep = 0, em = 0;
            for (int k = 0; k < n; ++k) {
                dh += P[i * n + k] * Dv[k * n + j];
                ep += Ip[i * n + k] * R[k * n + j];
                em += Im[i * n + k] * R[k * n + j];
            }
            T->Dhat[i * n + j] = (double)dh;
            T->Ep[i * n + j] = (double)ep;
            T->Em[i * n + j] = (double)em;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            T->RT[i * n + j] = T->R[j * n + i];
            T->PT[i * n + j] = T->P[j * n + i];
            T->DhatT[i * n + j] = T->Dhat[j * n + i];
            T->EpT[i * n + j] = T->Ep[j * n + i];
            T->EmT[i * n + j] = T->Em[j * n + i];
        }
    return 0;
}

extern "C" int sedg_tables(int n, int family, double *out, int cap)
{
    sedg_level_tab T;
    if (!out || sedg_build_level(n, family, &T)) return -1;
    int need = 2 * n + 2 * n * n + 2 * n + 3 * n * n + 2 * n + 2 * n * n;
    if (cap < need) return -1;
    double *o = out;
    auto put = [&](const double *a, int cnt) { std::memcpy(o, a, sizeof(double) * cnt); o += cnt; };
    put(T.xi, n); put(T.w, n); put(T.Dcal, n * n); put(T.D, n * n);
    put(T.bm, n); put(T.bp, n); put(T.P, n * n); put(T.R, n * n); put(T.Dhat, n * n);
    put(T.Bhl, n); put(T.Bhr, n); put(T.Ip, n * n); put(T.Im, n * n);
    return (int)(o - out);
}

// Refinement, coarsening and mortar tables of level n (App., non-conforming interfaces):
// Z = P^(n -> 2n) and Q = P^(n -> n/2), the projections of n nodal values onto 2n and n/2
// equal subcell means of [-1/2, 1/2] (Sec. 2.3 with other subcell counts), by exact
// integration of the monomial form of l_j; the L2-projection matrices of the mortar
// flux, L_+-_ij = l_i(xi_j / 2 +- 1/4) w_j / (2 w_i).
int sedg_build_nc(int n, int family, sedg_nc_tab *T)
{
    if (n < 2 || n > MAXN || (n & (n - 1))) return -1;
    q x[MAXN], w[MAXN];
    if (family == 1) lobatto(n, x, w);
    else gauss(n, x, w);
    q coef[MAXN][MAXN];
    for (int j = 0; j < n; ++j) lagrange_monomial(n, x, j, coef[j]);
    std::memset(T, 0, sizeof(*T));
    T->n = n;
    const int nz = 2 * n, nq = n / 2;
    for (int i = 0; i < nz; ++i)
        for (int j = 0; j < n; ++j) {
            q a = -q(1) / 2 + q(i) / nz, b = -q(1) / 2 + q(i + 1) / nz;
            T->Z[i * n + j] = (double)(nz * polyint(n, coef[j], a, b));
        }
    for (int i = 0; i < nq; ++i)
        for (int j = 0; j < n; ++j) {
            q a = -q(1) / 2 + q(i) / nq, b = -q(1) / 2 + q(i + 1) / nq;
            T->Q[i * n + j] = (double)(nq * polyint(n, coef[j], a, b));
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            q f = w[j] / (2 * w[i]);
            T->Lm[i * n + j] = (double)(polyval(n, coef[i], x[j] / 2 - q(1) / 4) * f);
            T->Lp[i * n + j] = (double)(polyval(n, coef[i], x[j] / 2 + q(1) / 4) * f);
        }
    return 0;
}

extern "C" int sedg_nc_tables(int n, int family, double *out, int cap)
{
    sedg_nc_tab T;
    if (!out || sedg_build_nc(n, family, &T)) return -1;
    int need = 2 * n * n + (n / 2) * n + 2 * n * n;
    if (cap < need) return -1;
    double *o = out;
    auto put = [&](const double *a, int cnt) { std::memcpy(o, a, sizeof(double) * cnt); o += cnt; };
    put(T.Z, 2 * n * n); put(T.Q, (n / 2) * n); put(T.Lm, n * n); put(T.Lp, n * n);
    return (int)(o - out);
}
