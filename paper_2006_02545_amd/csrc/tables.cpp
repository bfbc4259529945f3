// tables.cpp -- host-side reference data (Section 2 of the paper) and Gauss
// rules for the near-field correction library.
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "koorn.hpp"

namespace nfq {

namespace {

// LU factorisation with partial pivoting, A (n x n, row-major) in place.
bool lu_factor(int n, std::vector<long double> &A, std::vector<int> &piv)
{
    piv.resize(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        long double best = std::fabs(A[k * n + k]);
        for (int r = k + 1; r < n; ++r) {
            long double v = std::fabs(A[r * n + k]);
            if (v > best) { best = v; p = r; }
        }
        piv[k] = p;
        if (best == 0.0L) return false;
        if (p != k)
            for (int c = 0; c < n; ++c) std::swap(A[k * n + c], A[p * n + c]);
        for (int r = k + 1; r < n; ++r) {
            A[r * n + k] /= A[k * n + k];
            const long double f = A[r * n + k];
            for (int c = k + 1; c < n; ++c) A[r * n + c] -= f * A[k * n + c];
        }
    }
    return true;
}

void lu_solve(int n, const std::vector<long double> &LU, const std::vector<int> &piv,
              std::vector<long double> &b)
{
    for (int k = 0; k < n; ++k) std::swap(b[k], b[piv[k]]);
    for (int r = 1; r < n; ++r)
        for (int c = 0; c < r; ++c) b[r] -= LU[r * n + c] * b[c];
    for (int r = n - 1; r >= 0; --r) {
        for (int c = r + 1; c < n; ++c) b[r] -= LU[r * n + c] * b[c];
        b[r] /= LU[r * n + r];
    }
}

// Largest singular value of A (n x n) by power iteration on A^T A.
double spectral_norm(int n, const std::vector<double> &A)
{
    std::vector<long double> x(n, 1.0L), y(n), z(n);
    for (int i = 0; i < n; ++i) x[i] = 1.0L + 0.01L * i;
    long double lam = 0.0L;
    for (int it = 0; it < 20000; ++it) {
        for (int i = 0; i < n; ++i) {
            long double s = 0.0L;
            for (int j = 0; j < n; ++j) s += (long double)A[i * n + j] * x[j];
            y[i] = s;
        }
        for (int j = 0; j < n; ++j) {
            long double s = 0.0L;
            for (int i = 0; i < n; ++i) s += (long double)A[i * n + j] * y[i];
            z[j] = s;
        }
        long double nz = 0.0L;
        for (int j = 0; j < n; ++j) nz += z[j] * z[j];
        nz = std::sqrt(nz);
        long double nx = 0.0L;
        for (int j = 0; j < n; ++j) nx += x[j] * x[j];
        const long double newlam = nz / std::sqrt(nx);
        for (int j = 0; j < n; ++j) x[j] = z[j] / nz;
        if (it > 50 && std::fabs(newlam - lam) <= 1e-17L * newlam) { lam = newlam; break; }
        lam = newlam;
    }
    return (double)std::sqrt(lam);
}

// Eigenvalues and first eigenvector components of the symmetric tridiagonal
// matrix (diag d, off-diagonal e[0..n-2]) by the implicit QL method with
// Wilkinson-type shifts; z holds the first row of the eigenvector matrix.
void tridiag_ql(int n, std::vector<long double> &d, std::vector<long double> &e,
                std::vector<long double> &z)
{
    e.resize(n);
    e[n - 1] = 0.0L;
    z.assign(n, 0.0L);
    z[0] = 1.0L;
    for (int l = 0; l < n; ++l) {
        for (int iter = 0; iter < 200; ++iter) {
            int m = l;
            for (; m < n - 1; ++m) {
                const long double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-30L * dd || std::fabs(e[m]) < 1e-300L) break;
            }
            if (m == l) break;
            long double g = (d[l + 1] - d[l]) / (2.0L * e[l]);
            long double r = std::hypot(g, 1.0L);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            long double s = 1.0L, c = 1.0L, p = 0.0L;
            int i = m - 1;
            for (; i >= l; --i) {
                long double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0L) {
                    d[i + 1] -= p;
                    e[m] = 0.0L;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0L * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                // rotate the first row of the eigenvector matrix
                f = z[i + 1];
                z[i + 1] = s * z[i] + c * f;
                z[i] = c * z[i] - s * f;
            }
            if (r == 0.0L && i >= l) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0L;
        }
    }
}

}  // namespace

void gauss_rule(int n, int a, int b, std::vector<double> &y, std::vector<double> &w)
{
    // Jacobi polynomials on [-1,1] with weight (1-x)^a (1+x)^b; y = (1+x)/2
    // gives the weight 2^{a+b} (1-y)^a y^b on [0,1].
    std::vector<long double> dg(n), of(n > 1 ? n - 1 : 1), z;
    const long double A = a, B = b;
    for (int k = 0; k < n; ++k) {
        const long double s = 2.0L * k + A + B;
        if (k == 0)
            dg[k] = (B - A) / (A + B + 2.0L);
        else
            dg[k] = (B * B - A * A) / (s * (s + 2.0L));
        if (k + 1 < n) {
            const long double k1 = k + 1.0L, s1 = 2.0L * k1 + A + B;
            of[k] = std::sqrt(4.0L * k1 * (k1 + A) * (k1 + B) * (k1 + A + B)
                              / (s1 * s1 * (s1 + 1.0L) * (s1 - 1.0L)));
        }
    }
    std::vector<long double> e(of.begin(), of.end());
    tridiag_ql(n, dg, e, z);
    // mu0 = int_{-1}^{1} (1-x)^a (1+x)^b dx = 2^{a+b+1} a! b! / (a+b+1)!
    long double mu0 = std::pow(2.0L, A + B + 1.0L) * std::tgamma(A + 1.0L) * std::tgamma(B + 1.0L)
                      / std::tgamma(A + B + 2.0L);
    std::vector<std::pair<long double, long double>> nw(n);
    for (int i = 0; i < n; ++i) nw[i] = {dg[i], mu0 * z[i] * z[i]};
    std::sort(nw.begin(), nw.end());
    y.resize(n);
    w.resize(n);
    const long double scale = std::pow(2.0L, A + B + 1.0L);
    for (int i = 0; i < n; ++i) {
        y[i] = (double)((nw[i].first + 1.0L) / 2.0L);
        w[i] = (double)(nw[i].second / scale);
    }
}

void conical_rule(int ng, std::vector<double> &uvw)
{
    std::vector<double> xl, wl, yj, wj;
    gauss_rule(ng, 0, 0, xl, wl);
    gauss_rule(ng, 1, 0, yj, wj);
    uvw.resize(3 * ng * ng);
    int q = 0;
    for (int i = 0; i < ng; ++i)
        for (int k = 0; k < ng; ++k) {
            uvw[3 * q + 0] = xl[k] * (1.0 - yj[i]);
            uvw[3 * q + 1] = yj[i];
            uvw[3 * q + 2] = wl[k] * wj[i];
            ++q;
        }
}

std::string build_reference(int d, const double *uv, const double *w_in, RefData &out)
{
    if (d < 1 || d > 8) return "degree outside 1..8";
    const int nd = nd_of(d);
    for (int j = 0; j < nd; ++j) {
        const double u = uv[2 * j], v = uv[2 * j + 1];
        if (!(u > 0.0 && v > 0.0 && u + v < 1.0)) return "reference node not strictly inside T0";
    }
    // M[l][a] = K_a(node_l): node values = M * coefficients; V = M^{-1}.
    std::vector<long double> M(nd * nd);
    std::vector<double> Md(nd * nd);
    for (int l = 0; l < nd; ++l)
        koorn_visit_rt(d, uv[2 * l], uv[2 * l + 1], [&](int a, double K, double, double) {
            M[l * nd + a] = K;
            Md[l * nd + a] = K;
        });
    std::vector<int> piv;
    std::vector<long double> LU = M;
    if (!lu_factor(nd, LU, piv)) return "reference nodes not unisolvent (singular U)";
    out.d = d;
    out.nd = nd;
    out.uv.assign(uv, uv + 2 * nd);
    out.V.assign(nd * nd, 0.0);
    std::vector<long double> col(nd);
    for (int l = 0; l < nd; ++l) {
        std::fill(col.begin(), col.end(), 0.0L);
        col[l] = 1.0L;
        lu_solve(nd, LU, piv, col);
        for (int a = 0; a < nd; ++a) out.V[a * nd + l] = (double)col[a];
    }
    out.normV = spectral_norm(nd, out.V);
    out.cond = out.normV * spectral_norm(nd, Md);
    if (!(out.cond < 1e12)) return "reference nodes ill-conditioned (cond(U) > 1e12)";
    out.w.resize(nd);
    for (int l = 0; l < nd; ++l)
        out.w[l] = w_in ? w_in[l] : out.V[0 * nd + l] / std::sqrt(2.0);
    // differentiation matrices by projection; the conical rule with d + 2
    // points is exact for the degree 2d - 1 products
    std::vector<double> rule;
    conical_rule(d + 2, rule);
    std::vector<long double> Du(nd * nd, 0.0L), Dv(nd * nd, 0.0L);
    std::vector<double> K(nd), Ku(nd), Kv(nd);
    for (size_t q = 0; q < rule.size() / 3; ++q) {
        koorn_visit_rt(d, rule[3 * q], rule[3 * q + 1], [&](int a, double k, double ku, double kv) {
            K[a] = k;
            Ku[a] = ku;
            Kv[a] = kv;
        });
        const long double w = rule[3 * q + 2];
        for (int a = 0; a < nd; ++a)
            for (int m = 0; m < nd; ++m) {
                Du[a * nd + m] += w * Ku[a] * K[m];
                Dv[a * nd + m] += w * Kv[a] * K[m];
            }
    }
    out.D.resize(2 * nd * nd);
    for (int i = 0; i < nd * nd; ++i) {
        out.D[i] = (double)Du[i];
        out.D[nd * nd + i] = (double)Dv[i];
    }
    return "";
}

}  // namespace nfq
