// Host-side 1D polynomial machinery (see basis1d.hpp).
//
// Roots are bracketed by sign changes of the three-term recurrence on a fine
// grid, bisected and polished by Newton steps; every basis function is kept
// as a scale and a list of roots so that evaluation never goes through
// monomial coefficients.
#include "basis1d.hpp"

#include <cmath>
#include <algorithm>

namespace sipg {

double ProductPoly::value(double x) const {
    if (mirror) x = 1.0 - x;
    double v = c;
    for (double r : roots) v *= (x - r);
    return v;
}

double ProductPoly::deriv(double x) const {
    const double sgn = mirror ? -1.0 : 1.0;
    if (mirror) x = 1.0 - x;
    double s = 0.0;
    for (size_t k = 0; k < roots.size(); ++k) {
        double t = c;
        for (size_t l = 0; l < roots.size(); ++l)
            if (l != k) t *= (x - roots[l]);
        s += t;
    }
    return sgn * s;
}

// P_m^{(a,b)}(x) and its derivative by the standard recurrence in m.
static void jacobi_eval(int m, double a, double b, double x, double& p, double& dp) {
    double p0 = 1.0;
    if (m == 0) { p = 1.0; dp = 0.0; return; }
    double p1 = 0.5 * (a - b + (a + b + 2.0) * x);
    for (int k = 2; k <= m; ++k) {
        const double kk = k;
        const double s = 2.0 * kk + a + b;
        const double c1 = 2.0 * kk * (kk + a + b) * (s - 2.0);
        const double c2 = (s - 1.0) * (a * a - b * b);
        const double c3 = (s - 2.0) * (s - 1.0) * s;
        const double c4 = 2.0 * (kk + a - 1.0) * (kk + b - 1.0) * s;
        const double p2 = ((c2 + c3 * x) * p1 - c4 * p0) / c1;
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    // d/dx P_m^{(a,b)} = (m + a + b + 1)/2 * P_{m-1}^{(a+1,b+1)}
    double q, dq;
    jacobi_eval(m - 1, a + 1.0, b + 1.0, x, q, dq);
    dp = 0.5 * (m + a + b + 1.0) * q;
}

std::vector<double> jacobi_roots(int m, double a, double b) {
    std::vector<double> roots;
    if (m <= 0) return roots;
    const int grid = 20000;
    double xl = -1.0, pl, dpl;
    jacobi_eval(m, a, b, xl, pl, dpl);
    for (int i = 1; i <= grid && (int)roots.size() < m; ++i) {
        const double xr = -1.0 + 2.0 * i / grid;
        double pr, dpr;
        jacobi_eval(m, a, b, xr, pr, dpr);
        if (pr == 0.0) { roots.push_back(xr); xl = xr; pl = pr; continue; }
        if (pl * pr < 0.0) {
            double lo = xl, hi = xr, flo = pl;
            for (int it = 0; it < 200 && hi - lo > 1e-15; ++it) {
                const double mid = 0.5 * (lo + hi);
                double fm, dfm;
                jacobi_eval(m, a, b, mid, fm, dfm);
                if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
            }
            double x = 0.5 * (lo + hi);
            for (int it = 0; it < 3; ++it) {
                double f, df;
                jacobi_eval(m, a, b, x, f, df);
                if (df != 0.0) x -= f / df;
            }
            roots.push_back(x);
        }
        xl = xr;
        pl = pr;
    }
    std::sort(roots.begin(), roots.end());
    // exact symmetry for a == b
    if (a == b) {
        for (int i = 0; i < m / 2; ++i) {
            const double s = 0.5 * (roots[m - 1 - i] - roots[i]);
            roots[i] = -s;
            roots[m - 1 - i] = s;
        }
        if (m % 2 == 1) roots[m / 2] = 0.0;
    }
    return roots;
}

void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
    const std::vector<double> r = jacobi_roots(n, 0.0, 0.0);
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double p, dp;
        jacobi_eval(n, 0.0, 0.0, r[i], p, dp);
        x[i] = 0.5 * (r[i] + 1.0);
        w[i] = 0.5 * 2.0 / ((1.0 - r[i] * r[i]) * dp * dp);   // mapped to (0,1)
    }
}

std::vector<double> gauss_lobatto_points(int n) {
    std::vector<double> x(n);
    x[0] = 0.0;
    x[n - 1] = 1.0;
    const std::vector<double> r = jacobi_roots(n - 2, 1.0, 1.0);
    for (int i = 0; i < n - 2; ++i) x[i + 1] = 0.5 * (r[i] + 1.0);
    return x;
}

// Hermite-like basis of degree p (Section 4.1, Appendix A).
static std::vector<ProductPoly> hermite_like(int p) {
    std::vector<ProductPoly> f;
    if (p == 1) {
        f.push_back({-1.0, {1.0}, false});
        f.push_back({1.0, {0.0}, false});
        return f;
    }
    if (p == 2) {
        f.push_back({1.0, {1.0, 1.0}, false});
        f.push_back({-2.0, {0.0, 1.0}, false});
        f.push_back({1.0, {0.0, 0.0}, false});
        return f;
    }
    // interior nodes: roots of P^{4,4}_{p-3} mapped to (0,1)
    std::vector<double> nodes = jacobi_roots(p - 3, 4.0, 4.0);
    for (double& r : nodes) r = 0.5 * (r + 1.0);
    // g(xi) = (xi - 1)^2 prod (xi - r_l)
    ProductPoly g{1.0, {1.0, 1.0}, false};
    for (double r : nodes) g.roots.push_back(r);
    // free root of phi_0 from orthogonality of phi_0 = c0 (xi - s) g and
    // phi_1 = c1 xi g:  s = int xi^2 g^2 / int xi g^2 (exact with p+2 points)
    std::vector<double> xq, wq;
    gauss_rule(p + 2, xq, wq);
    double num = 0.0, den = 0.0;
    for (size_t q = 0; q < xq.size(); ++q) {
        const double gv = g.value(xq[q]);
        num += wq[q] * xq[q] * xq[q] * gv * gv;
        den += wq[q] * xq[q] * gv * gv;
    }
    const double s = num / den;
    const double g0 = g.value(0.0), dg0 = g.deriv(0.0);
    const double c0 = 1.0 / (-s * g0);                 // phi_0(0) = 1
    const double d0 = c0 * (g0 - s * dg0);             // phi_0'(0)
    const double c1 = -d0 / g0;                        // phi_1'(0) = -phi_0'(0)
    ProductPoly phi0{c0, {s}, false};
    ProductPoly phi1{c1, {0.0}, false};
    for (double r : g.roots) { phi0.roots.push_back(r); phi1.roots.push_back(r); }
    f.push_back(phi0);
    f.push_back(phi1);
    for (size_t m = 0; m < nodes.size(); ++m) {
        ProductPoly b{1.0, {0.0, 0.0, 1.0, 1.0}, false};
        for (size_t l = 0; l < nodes.size(); ++l)
            if (l != m) b.roots.push_back(nodes[l]);
        b.c = 1.0 / b.value(nodes[m]);
        f.push_back(b);
    }
    ProductPoly m1 = phi1; m1.mirror = true;
    ProductPoly m0 = phi0; m0.mirror = true;
    f.push_back(m1);
    f.push_back(m0);
    return f;
}

static std::vector<ProductPoly> nodal_gl(int p) {
    const std::vector<double> x = gauss_lobatto_points(p + 1);
    std::vector<ProductPoly> f;
    for (int j = 0; j <= p; ++j) {
        ProductPoly l{1.0, {}, false};
        double den = 1.0;
        for (int m = 0; m <= p; ++m)
            if (m != j) { l.roots.push_back(x[m]); den *= (x[j] - x[m]); }
        l.c = 1.0 / den;
        f.push_back(l);
    }
    return f;
}

// Lagrange basis in the p+1 Gauss points (collocated with the quadrature).
static std::vector<ProductPoly> nodal_gauss(int p) {
    std::vector<double> x, w;
    gauss_rule(p + 1, x, w);
    std::vector<ProductPoly> f;
    for (int j = 0; j <= p; ++j) {
        ProductPoly l{1.0, {}, false};
        double den = 1.0;
        for (int m = 0; m <= p; ++m)
            if (m != j) { l.roots.push_back(x[m]); den *= (x[j] - x[m]); }
        l.c = 1.0 / den;
        f.push_back(l);
    }
    return f;
}

std::vector<ProductPoly> make_basis(int kind, int p) {
    return kind == 0 ? hermite_like(p) : kind == 1 ? nodal_gl(p) : nodal_gauss(p);
}

// Gauss-Jordan inverse with partial pivoting (n <= 16).
static bool invert(int n, const std::vector<double>& A, std::vector<double>& Ai) {
    std::vector<double> M(A);
    Ai.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i) Ai[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
        if (M[piv * n + c] == 0.0) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(M[c * n + k], M[piv * n + k]);
                std::swap(Ai[c * n + k], Ai[piv * n + k]);
            }
        const double inv = 1.0 / M[c * n + c];
        for (int k = 0; k < n; ++k) { M[c * n + k] *= inv; Ai[c * n + k] *= inv; }
        for (int r = 0; r < n; ++r)
            if (r != c) {
                const double f = M[r * n + c];
                if (f == 0.0) continue;
                for (int k = 0; k < n; ++k) {
                    M[r * n + k] -= f * M[c * n + k];
                    Ai[r * n + k] -= f * Ai[c * n + k];
                }
            }
    }
    return true;
}

bool build_tables(int kind, int p, Tables1D& t) {
    const int n = p + 1;
    t.n = n;
    gauss_rule(n, t.points, t.weights);
    const std::vector<ProductPoly> f = make_basis(kind, p);
    t.S.assign(n * n, 0.0);
    t.Sg.assign(n * n, 0.0);
    for (int q = 0; q < n; ++q)
        for (int j = 0; j < n; ++j) {
            t.S[q * n + j] = f[j].value(t.points[q]);
            t.Sg[q * n + j] = f[j].deriv(t.points[q]);
        }
    // collocation derivative: Lagrange polynomials in the Gauss points, via
    // barycentric weights lambda_j = 1 / prod_{m != j} (x_j - x_m)
    std::vector<double> lam(n, 1.0);
    for (int j = 0; j < n; ++j)
        for (int m = 0; m < n; ++m)
            if (m != j) lam[j] /= (t.points[j] - t.points[m]);
    t.D.assign(n * n, 0.0);
    for (int q = 0; q < n; ++q) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j)
            if (j != q) {
                const double v = (lam[j] / lam[q]) / (t.points[q] - t.points[j]);
                t.D[q * n + j] = v;
                diag -= v;
            }
        t.D[q * n + q] = diag;
    }
    t.v0.resize(n); t.g0.resize(n); t.v1.resize(n); t.g1.resize(n);
    for (int j = 0; j < n; ++j) {
        t.v0[j] = f[j].value(0.0);
        t.g0[j] = f[j].deriv(0.0);
        t.v1[j] = f[j].value(1.0);
        t.g1[j] = f[j].deriv(1.0);
    }
    const std::vector<double> xgl = gauss_lobatto_points(n);
    t.E.assign(n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) t.E[i * n + j] = f[i].value(xgl[j]);
    return invert(n, t.E, t.T);
}

bool child_embedding(int kind, int p, double a, std::vector<double>& M0, std::vector<double>& M1) {
    const int n = p + 1;
    const std::vector<ProductPoly> f = make_basis(kind, p);
    const std::vector<double> x = gauss_lobatto_points(n);   // n distinct points
    // V[m][i] = phi_i(x_m); C_s[m][j] = phi_j(o_s + l_s x_m) with child 0 on
    // [0, a] and child 1 on [a, 1]; M_s = V^-1 C_s
    std::vector<double> V(n * n), Vi;
    for (int m = 0; m < n; ++m)
        for (int i = 0; i < n; ++i) V[m * n + i] = f[i].value(x[m]);
    if (!invert(n, V, Vi)) return false;
    for (int s = 0; s < 2; ++s) {
        const double o = s == 0 ? 0.0 : a, l = s == 0 ? a : 1.0 - a;
        std::vector<double>& M = s == 0 ? M0 : M1;
        M.assign(n * n, 0.0);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int m = 0; m < n; ++m) acc += Vi[i * n + m] * f[j].value(o + l * x[m]);
                M[i * n + j] = acc;
            }
    }
    return true;
}

bool degree_embedding(int kind, int pf, int pc, std::vector<double>& E) {
    const int nf = pf + 1, nc = pc + 1;
    if (pc > pf || pc < 1) return false;
    const std::vector<ProductPoly> ff = make_basis(kind, pf), fc = make_basis(kind, pc);
    const std::vector<double> x = gauss_lobatto_points(nf);   // nf distinct points
    // V[m][i] = phi^f_i(x_m); C[m][j] = phi^c_j(x_m); E = V^-1 C (nf x nc)
    std::vector<double> V(nf * nf), Vi;
    for (int m = 0; m < nf; ++m)
        for (int i = 0; i < nf; ++i) V[m * nf + i] = ff[i].value(x[m]);
    if (!invert(nf, V, Vi)) return false;
    E.assign(nf * nc, 0.0);
    for (int i = 0; i < nf; ++i)
        for (int j = 0; j < nc; ++j) {
            double acc = 0.0;
            for (int m = 0; m < nf; ++m) acc += Vi[i * nf + m] * fc[j].value(x[m]);
            E[i * nc + j] = acc;
        }
    return true;
}

// Generalized symmetric-definite eigenproblem L y = lambda M y of size m
// (row major): Cholesky M = C C^T, the symmetric C^-1 L C^-T diagonalized by
// cyclic Jacobi rotations, y = C^-T (rotations).  Columns of Y are the
// eigenvectors, Y^T M Y = I.
static bool sym_gen_eig(int m, const std::vector<double>& L, const std::vector<double>& M,
                        std::vector<double>& Y, std::vector<double>& lam) {
    std::vector<double> C(m * m, 0.0);
    for (int j = 0; j < m; ++j) {
        double d = M[j * m + j];
        for (int k = 0; k < j; ++k) d -= C[j * m + k] * C[j * m + k];
        if (!(d > 0.0)) return false;
        C[j * m + j] = std::sqrt(d);
        for (int i = j + 1; i < m; ++i) {
            double v = M[i * m + j];
            for (int k = 0; k < j; ++k) v -= C[i * m + k] * C[j * m + k];
            C[i * m + j] = v / C[j * m + j];
        }
    }
    std::vector<double> Ci;
    if (!invert(m, C, Ci)) return false;
    std::vector<double> B(m * m, 0.0), W(m * m, 0.0), R(m * m, 0.0);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            double v = 0.0;
            for (int k = 0; k < m; ++k) v += Ci[i * m + k] * L[k * m + j];
            W[i * m + j] = v;
        }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            double v = 0.0;
            for (int k = 0; k < m; ++k) v += W[i * m + k] * Ci[j * m + k];
            B[i * m + j] = v;
        }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < i; ++j) B[i * m + j] = B[j * m + i] = 0.5 * (B[i * m + j] + B[j * m + i]);
    for (int i = 0; i < m; ++i) R[i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                tot += B[i * m + j] * B[i * m + j];
                if (i != j) off += B[i * m + j] * B[i * m + j];
            }
        if (off <= 1e-32 * tot) break;
        for (int pp = 0; pp < m - 1; ++pp)
            for (int qq = pp + 1; qq < m; ++qq) {
                const double apq = B[pp * m + qq];
                if (apq == 0.0) continue;
                const double theta = (B[qq * m + qq] - B[pp * m + pp]) / (2.0 * apq);
                const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(tt * tt + 1.0), sn = tt * c;
                for (int k = 0; k < m; ++k) {   // B <- B G (columns p, q)
                    const double bkp = B[k * m + pp], bkq = B[k * m + qq];
                    B[k * m + pp] = c * bkp - sn * bkq;
                    B[k * m + qq] = sn * bkp + c * bkq;
                }
                for (int k = 0; k < m; ++k) {   // B <- G^T B (rows p, q)
                    const double bpk = B[pp * m + k], bqk = B[qq * m + k];
                    B[pp * m + k] = c * bpk - sn * bqk;
                    B[qq * m + k] = sn * bpk + c * bqk;
                }
                for (int k = 0; k < m; ++k) {   // R <- R G
                    const double rkp = R[k * m + pp], rkq = R[k * m + qq];
                    R[k * m + pp] = c * rkp - sn * rkq;
                    R[k * m + qq] = sn * rkp + c * rkq;
                }
            }
    }
    Y.assign(m * m, 0.0);
    lam.assign(m, 0.0);
    for (int e = 0; e < m; ++e) {
        lam[e] = B[e * m + e];
        for (int j = 0; j < m; ++j) {
            double v = 0.0;
            for (int k = 0; k < m; ++k) v += Ci[k * m + j] * R[k * m + e];
            Y[j * m + e] = v;
        }
    }
    return true;
}

// Separable block-Jacobi preconditioner (Section 6.4): the 1D SIPG stiffness
// matrix L of an element with two interior faces and the 1D mass matrix M on
// the unit interval (Gauss quadrature with n points is exact for both),
// penalty eta (p+1)^2.  Both commute with the reflection xi -> 1 - xi (the
// bases are symmetric, phi_{p-i}(xi) = phi_i(1 - xi)), so the eigenvectors
// of L z = lambda M z are solved for separately on the reflection-even
// vectors (h = n/2 pairs u_j = u_{n-1-j}, plus the middle entry for odd n)
// and the reflection-odd ones (u_j = -u_{n-1-j}).  Output order: the
// ceil(n/2) even eigenvectors, then the floor(n/2) odd ones.
bool fdm_1d(int kind, int p, double eta, std::vector<double>& Zt, std::vector<double>& lam,
            std::vector<double>* packed) {
    Tables1D t;
    if (!build_tables(kind, p, t)) return false;
    const int n = p + 1, h = n / 2, ne = n - h, no = h;
    const double sigma = eta * double(n) * double(n);
    std::vector<double> L(n * n, 0.0), M(n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double l = 0.0, m = 0.0;
            for (int q = 0; q < n; ++q) {
                l += t.weights[q] * t.Sg[q * n + i] * t.Sg[q * n + j];
                m += t.weights[q] * t.S[q * n + i] * t.S[q * n + j];
            }
            // face at 0 (outward normal -1) and at 1 (outward normal +1):
            // sigma u v - 1/2 v (n u') - 1/2 (n v') u
            l += sigma * t.v0[i] * t.v0[j] + 0.5 * (t.v0[i] * t.g0[j] + t.g0[i] * t.v0[j]);
            l += sigma * t.v1[i] * t.v1[j] - 0.5 * (t.v1[i] * t.g1[j] + t.g1[i] * t.v1[j]);
            L[i * n + j] = l;
            M[i * n + j] = m;
        }
    // parity bases: even column e (e < h: unit vectors j and n-1-j; e = h for
    // odd n: the middle), odd column o (unit j minus unit n-1-j)
    auto basis_vec = [&](bool even, int e, std::vector<double>& v) {
        v.assign(n, 0.0);
        if (even && e == h) { v[h] = 1.0; return; }
        v[e] = 1.0;
        v[n - 1 - e] = even ? 1.0 : -1.0;
    };
    Zt.assign(n * n, 0.0);
    lam.assign(n, 0.0);
    if (packed) packed->assign(ne * (h + 1) + no * h, 0.0);
    int row = 0;
    for (int par = 0; par < 2; ++par) {
        const bool even = par == 0;
        const int m = even ? ne : no;
        if (m == 0) continue;
        std::vector<std::vector<double>> P(m);
        for (int e = 0; e < m; ++e) basis_vec(even, e, P[e]);
        std::vector<double> Lr(m * m), Mr(m * m), Y, lr;
        for (int a = 0; a < m; ++a)
            for (int b2 = 0; b2 < m; ++b2) {
                double l = 0.0, mm = 0.0;
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        l += P[a][i] * L[i * n + j] * P[b2][j];
                        mm += P[a][i] * M[i * n + j] * P[b2][j];
                    }
                Lr[a * m + b2] = l;
                Mr[a * m + b2] = mm;
            }
        if (!sym_gen_eig(m, Lr, Mr, Y, lr)) return false;
        for (int e = 0; e < m; ++e, ++row) {
            lam[row] = lr[e];
            for (int j = 0; j < n; ++j) {
                double v = 0.0;
                for (int a = 0; a < m; ++a) v += P[a][j] * Y[a * m + e];
                Zt[row * n + j] = v;
            }
            if (packed) {
                // coefficients of the reduced basis: y[j] for j < h, middle y[h]
                if (even) for (int a = 0; a < m; ++a) (*packed)[e * (h + 1) + a] = Y[a * m + e];
                else for (int a = 0; a < m; ++a) (*packed)[ne * (h + 1) + e * h + a] = Y[a * m + e];
            }
        }
    }
    return true;
}

}  // namespace sipg
