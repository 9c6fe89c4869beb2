// Host-side 1D polynomial machinery for the operator set-up: Jacobi roots,
// Gauss and Gauss-Lobatto rules, the Hermite-like basis of Section 4.1 and
// the nodal Gauss-Lobatto basis, all in double precision and in product form.
#pragma once

#include <vector>

namespace sipg {

// p(xi) = c * prod_l (xi - r_l); `mirror` evaluates p(1 - xi) instead.
struct ProductPoly {
    double c = 1.0;
    std::vector<double> roots;
    bool mirror = false;
    double value(double x) const;
    double deriv(double x) const;
};

// Roots of the Jacobi polynomial P_m^{(a,b)} on (-1,1), ascending.
std::vector<double> jacobi_roots(int m, double a, double b);

// Gauss-Legendre rule with n points on (0,1).
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w);

// The n Gauss-Lobatto points on [0,1].
std::vector<double> gauss_lobatto_points(int n);

// Degree-p 1D basis: 0 = Hermite-like, 1 = nodal Gauss-Lobatto Lagrange,
// 2 = nodal Gauss Lagrange.
std::vector<ProductPoly> make_basis(int kind, int p);

// All 1D tables (see sipg_host_tables in sipg.h), n = p + 1, row major.
struct Tables1D {
    int n = 0;
    std::vector<double> points, weights;
    std::vector<double> S, Sg, D;          // S[q][j], S'[q][j], D[q][j]
    std::vector<double> v0, g0, v1, g1;    // face values/derivatives at 0 and 1
    std::vector<double> T;                 // E^-1, E[i][j] = phi_i(x^GL_j)
    std::vector<double> E;
};
bool build_tables(int kind, int p, Tables1D& t);

// Embedding of the coarse 1D space into the two children [0, a] and [a, 1]
// of a coarse interval: phi_j(a xi) = sum_i M_0[i][j] phi_i(xi) and
// phi_j(a + (1 - a) xi) = sum_i M_1[i][j] phi_i(xi) (row major, n x n; a = 1/2
// for two halves).  Exact: both sides are polynomials of degree p.
bool child_embedding(int kind, int p, double a, std::vector<double>& M0, std::vector<double>& M1);

// Embedding of the degree-pc space into the degree-pf space (pc <= pf) of
// the same basis kind on one interval: phi^pc_j = sum_i E[i][j] phi^pf_i
// (row major, (pf+1) x (pc+1)).  Exact: interpolation in pf+1 points.
bool degree_embedding(int kind, int pf, int pc, std::vector<double>& E);

// 1D matrices of the separable block preconditioner of Section 6.4 (eq.
// KDlaplace_dg) on the unit interval, penalty eta (p+1)^2, interior element:
// generalized eigenvectors (rows of Zt) and eigenvalues of L z = lambda M z,
// with Z^T M Z = I; the ceil(n/2) reflection-even eigenvectors first, then
// the reflection-odd ones.  `packed` (optional) receives the parity-split
// form the device uses: for each even vector its entries 0..h (h = n/2; entry
// h is the middle one, zero for even n), then for each odd vector its
// entries 0..h-1.
bool fdm_1d(int kind, int p, double eta, std::vector<double>& Zt, std::vector<double>& lam,
            std::vector<double>* packed = nullptr);

}  // namespace sipg
