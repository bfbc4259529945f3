/*
 * nfq_oracle.c -- plain, slow CPU oracle for the near-field quadrature
 * correction generator of Greengard, O'Neil, Rachh, Vico, "Fast multipole
 * methods for the evaluation of layer potentials with locally-corrected
 * quadratures" (arXiv 2006.02545).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP path: its own Koornwinder evaluation (explicit Jacobi sums),
 * its own Gauss rules (root bracketing + Newton on explicit sums), its own
 * matrix inverse and spectral norm, its own adaptive integrators.
 *
 * What it computes, for every target x and every patch Gamma_j in the dual
 * list T_eta(x) (Section 4, near-field definitions), plus the target's own
 * patch when the target is a node (self interaction, Section 4 opening):
 *
 *     a^j_l(x) = sum_{nm} V_(nm),l I^j_nm(x)                       (Sec. 4.3)
 *     I^j_nm(x) = int_T0 K(x, X^j(u,v)) K_nm(u,v) [J] du dv
 *
 * with the kernel  alpha * G_k(r) J + beta * n(y).grad_y G_k(x,y)
 * (single layer, double layer, Section 3), n = X_u x X_v unnormalised
 * (Section 3.1), G_k = exp(ikr)/(4 pi r) (Section 1).
 *
 * Two modes:
 *  - METHOD: the paper's adaptive scheme (Section 4.3): a rule on T0,
 *    1->4 midpoint subdivision, accept the children when
 *    ||I_T - sum I_C||_2 <= tau |T|/|T0|, tau = loosen * eps * d_j / ||V||_2
 *    (scaled tolerance of Section 4.2, eq. for q_j, and Section 4.3).
 *    Subtriangle rule: conical product (Gauss-Jacobi(1,0) x Gauss-Legendre),
 *    n_g points per direction (8 by default), standing in for the unprinted
 *    q-th order Vioreanu-Rokhlin rule.  A test whose difference is below
 *    the estimated double-precision rounding level of the moments is also
 *    accepted (near a target the scaled threshold of deep subtriangles can
 *    fall below that level, and refining further cannot help).
 *  - TRUTH: the same integrals to ~1e-13 relative (20-point rules, tight
 *    tolerance, deep trees) for parity checks.
 *  Self patches (both modes): the target splits T0 into three triangles,
 *  each Duffy-collapsed at the target, integrated by nested adaptive
 *  Gauss-Legendre (stands in for the unprinted generalized Gaussian tables,
 *  Section 4 opening, error bound eq. errestself).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#undef I
#define IU _Complex_I

typedef double complex cplx;

/* safety factor of the rounding-floor acceptance of the adaptive test */
#ifndef ORC_NOISE_KAPPA
#define ORC_NOISE_KAPPA 16.0
#endif
typedef __float128 qreal;

#define ORC_MAXD 12
#define ORC_MAXND ((ORC_MAXD + 1) * (ORC_MAXD + 2) / 2)
#define ORC_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------ */
/* Small helpers                                                       */
/* ------------------------------------------------------------------ */

static long double binom_direct(int n, int k)
{
    if (k < 0 || k > n) return 0.0L;
    long double r = 1.0L;
    for (int i = 1; i <= k; ++i) r = r * (long double)(n - k + i) / (long double)i;
    return r;
}

/* table of binomial coefficients C(n,k), n < 96 */
static long double g_binom[96][96];
static int g_binom_ok = 0;

static long double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0L;
    if (n >= 96) return binom_direct(n, k);
    if (!g_binom_ok) {
        for (int a = 0; a < 96; ++a)
            for (int b = 0; b < 96; ++b) g_binom[a][b] = binom_direct(a, b);
        g_binom_ok = 1;
    }
    return g_binom[n][k];
}

/* x^e with the convention 0^0 = 1; e < 0 only ever multiplies a zero
 * coefficient, return 0 then. */
static double ipow(double x, int e)
{
    if (e < 0) return 0.0;
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

static long double ipowl_(long double x, int e)
{
    if (e < 0) return 0.0L;
    long double r = 1.0L;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

int orc_nd(int d) { return (d + 1) * (d + 2) / 2; }

/* ------------------------------------------------------------------ */
/* Jacobi polynomials by the explicit finite sum                       */
/*   P_n^{(a,b)}(x) = sum_s C(n+a, n-s) C(n+b, s) ((x-1)/2)^s ((x+1)/2)^{n-s}
 * (textbook; Szego 4.3.2).  Derivative: d/dx P_n^{(a,b)} =
 * (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}.                                      */
/* ------------------------------------------------------------------ */
static long double jacobi_l(int n, int a, int b, long double x)
{
    if (n < 0) return 0.0L;
    long double t1 = (x - 1.0L) / 2.0L, t2 = (x + 1.0L) / 2.0L, s = 0.0L;
    for (int k = 0; k <= n; ++k)
        s += binom(n + a, n - k) * binom(n + b, k) * ipowl_(t1, k) * ipowl_(t2, n - k);
    return s;
}

static long double jacobi_dl(int n, int a, int b, long double x)
{
    if (n <= 0) return 0.0L;
    return 0.5L * (long double)(n + a + b + 1) * jacobi_l(n - 1, a + 1, b + 1, x);
}

/* ------------------------------------------------------------------ */
/* Koornwinder polynomials on T0 (Section 2):                          */
/*   K_nm(u,v) = c_nm (1-v)^m P^{(0,2m+1)}_{n-m}(1-2v) P_m((2u+v-1)/(1-v))
 * written without the division:                                       */
/*   P^{(0,b)}_k(1-2v) = sum_s C(k,k-s) C(k+b,s) (-v)^s (1-v)^{k-s}     */
/*   (1-v)^m P_m(xi)   = sum_s C(m,s)^2 (u+v-1)^s u^{m-s}               */
/* c_nm = sqrt(2 (n+1) (2m+1)) makes them orthonormal on T0 (pinned by */
/* the Gram-matrix test).  Index of (n,m) is n(n+1)/2 + m.             */
/* ------------------------------------------------------------------ */
static void koorn_ld(int d, long double u, long double v, long double *K, long double *Ku,
                     long double *Kv)
{
    for (int n = 0; n <= d; ++n) {
        for (int m = 0; m <= n; ++m) {
            int k = n - m, b = 2 * m + 1;
            long double A = 0.0L, Av = 0.0L;
            for (int s = 0; s <= k; ++s) {
                long double c = binom(k, k - s) * binom(k + b, s);
                A += c * ipowl_(-v, s) * ipowl_(1.0L - v, k - s);
                /* d/dv [(-v)^s (1-v)^(k-s)] */
                Av += c * (-(long double)s * ipowl_(-v, s - 1) * ipowl_(1.0L - v, k - s)
                           - (long double)(k - s) * ipowl_(-v, s) * ipowl_(1.0L - v, k - s - 1));
            }
            long double B = 0.0L, Bu = 0.0L, Bv = 0.0L, w = u + v - 1.0L;
            for (int s = 0; s <= m; ++s) {
                long double c = binom(m, s) * binom(m, s);
                B += c * ipowl_(w, s) * ipowl_(u, m - s);
                Bu += c * ((long double)s * ipowl_(w, s - 1) * ipowl_(u, m - s)
                           + (long double)(m - s) * ipowl_(w, s) * ipowl_(u, m - s - 1));
                Bv += c * (long double)s * ipowl_(w, s - 1) * ipowl_(u, m - s);
            }
            long double cn = sqrtl(2.0L * (n + 1) * (2 * m + 1));
            int idx = n * (n + 1) / 2 + m;
            if (K) K[idx] = cn * A * B;
            if (Ku) Ku[idx] = cn * A * Bu;
            if (Kv) Kv[idx] = cn * (Av * B + A * Bv);
        }
    }
}

void orc_koornwinder(int d, double u, double v, double *K, double *Ku, double *Kv)
{
    long double a[ORC_MAXND], b[ORC_MAXND], c[ORC_MAXND];
    koorn_ld(d, u, v, a, b, c);
    for (int i = 0; i < orc_nd(d); ++i) {
        if (K) K[i] = (double)a[i];
        if (Ku) Ku[i] = (double)b[i];
        if (Kv) Kv[i] = (double)c[i];
    }
}

/* ------------------------------------------------------------------ */
/* Gauss rules: roots of P_n^{(a,b)} bracketed on a fine grid, refined */
/* by bisection then Newton (long double).  Weights (Szego 15.3.5):    */
/*  w_i = G(n+a+1)G(n+b+1)/(G(n+a+b+1) n!) 2^{a+b+1}/((1-x_i^2) P'(x_i)^2) */
/* Returned on [0,1] for the weight (1-y)^a y^b: y = (1 - x)/2 ...     */
/* we map x in [-1,1] -> y = (x+1)/2, so (1-x)^a (1+x)^b = 2^{a+b}    */
/* (1-y)^a y^b and dx = 2 dy.                                          */
/* ------------------------------------------------------------------ */
int orc_gauss_jacobi(int n, int a, int b, double *y, double *w)
{
    if (n < 1 || n > 64) return -1;
    int M = 40000, found = 0;
    long double prevx = -1.0L, prevf = jacobi_l(n, a, b, -1.0L);
    long double roots[64];
    for (int i = 1; i <= M && found < n; ++i) {
        long double x = -1.0L + 2.0L * (long double)i / (long double)M;
        long double f = jacobi_l(n, a, b, x);
        if ((prevf < 0 && f > 0) || (prevf > 0 && f < 0) || f == 0.0L) {
            long double lo = prevx, hi = x, flo = prevf;
            for (int it = 0; it < 200; ++it) {
                long double mid = 0.5L * (lo + hi), fm = jacobi_l(n, a, b, mid);
                if ((flo < 0 && fm < 0) || (flo > 0 && fm > 0)) { lo = mid; flo = fm; }
                else hi = mid;
            }
            long double r = 0.5L * (lo + hi);
            for (int it = 0; it < 3; ++it) {
                long double dp = jacobi_dl(n, a, b, r);
                if (dp != 0.0L) r -= jacobi_l(n, a, b, r) / dp;
            }
            roots[found++] = r;
            if (f == 0.0L) { x += 1e-12L; f = jacobi_l(n, a, b, x); }
        }
        prevx = x; prevf = f;
    }
    if (found != n) return -2;
    long double cst = expl(lgammal(n + a + 1) + lgammal(n + b + 1) - lgammal(n + a + b + 1)
                           - lgammal(n + 1)) * powl(2.0L, a + b + 1);
    for (int i = 0; i < n; ++i) {
        long double x = roots[i], dp = jacobi_dl(n, a, b, x);
        long double wx = cst / ((1.0L - x * x) * dp * dp);
        y[i] = (double)((x + 1.0L) / 2.0L);
        w[i] = (double)(wx / powl(2.0L, a + b + 1));
    }
    return 0;
}

/* Conical-product rule on T0 with ng^2 nodes, exact for total degree
 * <= 2 ng - 1:  v = y, u = x (1 - y), du dv = (1 - y) dx dy, with
 * Gauss-Jacobi (weight 1-y) in y and Gauss-Legendre in x.
 * Output uvw[3*i + {0,1,2}] = u, v, weight; weights sum to 1/2. */
int orc_conical_rule(int ng, double *uvw)
{
    double xg[64], wg[64], yj[64], wj[64];
    if (orc_gauss_jacobi(ng, 0, 0, xg, wg)) return -1;
    if (orc_gauss_jacobi(ng, 1, 0, yj, wj)) return -1;
    int q = 0;
    for (int i = 0; i < ng; ++i)
        for (int j = 0; j < ng; ++j) {
            uvw[3 * q + 0] = xg[j] * (1.0 - yj[i]);
            uvw[3 * q + 1] = yj[i];
            uvw[3 * q + 2] = wg[j] * wj[i];
            ++q;
        }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Dense linear algebra (long double): inverse by Gauss-Jordan with    */
/* partial pivoting; spectral norm by cyclic Jacobi eigenvalues of     */
/* V^T V.                                                              */
/* ------------------------------------------------------------------ */
static int invert_l(int n, long double *A, long double *Ai)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ai[i * n + j] = (i == j) ? 1.0L : 0.0L;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsl(A[r * n + c]) > fabsl(A[p * n + c])) p = r;
        if (A[p * n + c] == 0.0L) return -1;
        if (p != c)
            for (int j = 0; j < n; ++j) {
                long double t = A[c * n + j]; A[c * n + j] = A[p * n + j]; A[p * n + j] = t;
                t = Ai[c * n + j]; Ai[c * n + j] = Ai[p * n + j]; Ai[p * n + j] = t;
            }
        long double piv = A[c * n + c];
        for (int j = 0; j < n; ++j) { A[c * n + j] /= piv; Ai[c * n + j] /= piv; }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            long double f = A[r * n + c];
            if (f == 0.0L) continue;
            for (int j = 0; j < n; ++j) {
                A[r * n + j] -= f * A[c * n + j];
                Ai[r * n + j] -= f * Ai[c * n + j];
            }
        }
    }
    return 0;
}

static long double jacobi_eig_max(int n, long double *S)
{
    for (int sweep = 0; sweep < 100; ++sweep) {
        long double off = 0.0L;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += S[i * n + j] * S[i * n + j];
        if (off < 1e-40L) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                long double apq = S[p * n + q];
                if (fabsl(apq) < 1e-300L) continue;
                long double app = S[p * n + p], aqq = S[q * n + q];
                long double th = (aqq - app) / (2.0L * apq);
                long double t = (th >= 0 ? 1.0L : -1.0L) / (fabsl(th) + sqrtl(th * th + 1.0L));
                long double c = 1.0L / sqrtl(t * t + 1.0L), s = t * c;
                for (int k = 0; k < n; ++k) {
                    long double skp = S[k * n + p], skq = S[k * n + q];
                    S[k * n + p] = c * skp - s * skq;
                    S[k * n + q] = s * skp + c * skq;
                }
                for (int k = 0; k < n; ++k) {
                    long double spk = S[p * n + k], sqk = S[q * n + k];
                    S[p * n + k] = c * spk - s * sqk;
                    S[q * n + k] = s * spk + c * sqk;
                }
            }
    }
    long double mx = 0.0L;
    for (int i = 0; i < n; ++i) if (S[i * n + i] > mx) mx = S[i * n + i];
    return mx;
}

/* Per-degree reference data (Section 2): U_(nm),j = K_nm(u_j, v_j),
 * V = U^{-1} stored V[(nm) * nd + l], ||V||_2, interpolatory weights
 * w_l = int_T0 L_l = V_(00),l * int K_00 = V_(00),l / sqrt(2). */
typedef struct {
    int d, nd, ok;
    double uv[2 * ORC_MAXND];
    double V[ORC_MAXND * ORC_MAXND];
    double normV;
    double w[ORC_MAXND];
} orc_ref;

int orc_reference(int d, const double *uv, double *V, double *normV, double *w)
{
    int nd = orc_nd(d);
    long double *U = malloc(sizeof(long double) * nd * nd);
    long double *Vi = malloc(sizeof(long double) * nd * nd);
    long double *S = malloc(sizeof(long double) * nd * nd);
    double K[ORC_MAXND];
    for (int j = 0; j < nd; ++j) {
        orc_koornwinder(d, uv[2 * j], uv[2 * j + 1], K, NULL, NULL);
        for (int i = 0; i < nd; ++i) U[i * nd + j] = K[i];  /* row = (nm), col = node j */
    }
    int rc = invert_l(nd, U, Vi);   /* Vi[j][nm]: V = U^{-1} is (node x nm)?  see below */
    if (rc) { free(U); free(Vi); free(S); return -1; }
    /* U maps coefficients c (indexed by nm) to node values f_j = sum_nm U_(nm),j c_nm,
     * i.e. f = U^T c with U stored [nm][j].  The matrix that maps values to
     * coefficients is (U^T)^{-1}; as an array indexed [nm][l] it is the
     * transpose of inv(U^T), i.e. inv(U) read as [l][nm] -> we store
     * V[(nm), l] = Vi[l][nm] where Vi = inv(U) with U stored [nm][j].
     * Check: sum_l V[(nm),l] f_l = sum_l inv(U)[l][nm] f_l = (inv(U)^T f)[nm]
     *        = (inv(U^T) f)[nm] = c_nm.                                 */
    for (int a = 0; a < nd; ++a)
        for (int l = 0; l < nd; ++l) V[a * nd + l] = (double)Vi[l * nd + a];
    for (int i = 0; i < nd; ++i)
        for (int j = 0; j < nd; ++j) {
            long double s = 0.0L;
            for (int k = 0; k < nd; ++k) s += Vi[k * nd + i] * Vi[k * nd + j];
            S[i * nd + j] = s;
        }
    *normV = (double)sqrtl(jacobi_eig_max(nd, S));
    for (int l = 0; l < nd; ++l) w[l] = V[0 * nd + l] / sqrt(2.0);
    free(U); free(Vi); free(S);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Problem description (all host arrays)                               */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t P;
    const int32_t *degree;       /* [P] */
    const int64_t *node_ptr;     /* [P+1] */
    const double *xyz;           /* [N][3] */
    int64_t NT;
    const double *txyz;          /* [NT][3] */
    const int64_t *node_of_target; /* [NT], node id or -1 */
    const int64_t *near_row_ptr; /* [NT+1] */
    const int32_t *near_patch;   /* ascending per row, self excluded */
    const double *ref_uv[ORC_MAXD + 1];
    double alpha_re, alpha_im, beta_re, beta_im, k_re, k_im;
    double tol, loosen;
    int max_depth;   /* method mode */
    int ng;          /* method-mode rule size per direction (0 -> d + 2) */
    int mode;        /* 0 = method, 1 = truth */
    int pad;
} orc_problem;

typedef struct {
    int64_t visits;        /* rule evaluations on (sub)triangles, near pairs */
    int64_t checks;        /* parent-vs-children comparisons */
    int64_t nonconverged;  /* pairs that hit the depth limit */
    int64_t max_level;     /* deepest children level used */
    int64_t near_pairs;
    int64_t self_targets;
    int64_t self_evals;    /* integrand evaluations in self quadrature */
} orc_stats;

typedef struct {
    cplx alpha, beta, k;
} kern_t;

/* Geometry of one patch: chart coefficients x_nm = sum_l V_(nm),l x_l
 * (Section 3.2, Koornwinder approximation of the chart). */
typedef struct {
    int d, nd;
    long double coef[3][ORC_MAXND];
    const orc_ref *ref;
    double dj;   /* min_l sqrt(J(u_l,v_l) |w_l|) (Section 4.2) */
    double rho;  /* max_l |x_l|: coordinate scale of the patch */
} patch_t;

/* Chart X = sum_nm x_nm K_nm, its derivatives, n = X_u x X_v and J = |n|
 * at (u,v) (Section 3.1).  Carried in long double: the separations
 * x - X(y) and n(y).(x - X(y)) of near-singular integrands then have no
 * rounding floor at the level the adaptive tests look at.  Basis values
 * are returned (as double) in K. */
typedef struct { long double X[3], Xu[3], Xv[3], n[3], J; } geo_t;

static orc_ref g_ref[ORC_MAXD + 1];

static const orc_ref *get_ref(const orc_problem *pb, int d)
{
    orc_ref *r = &g_ref[d];
    const double *uv = pb->ref_uv[d];
    if (!uv) return NULL;
    if (r->ok && memcmp(r->uv, uv, sizeof(double) * 2 * orc_nd(d)) == 0) return r;
    r->d = d; r->nd = orc_nd(d);
    memcpy(r->uv, uv, sizeof(double) * 2 * r->nd);
    if (orc_reference(d, uv, r->V, &r->normV, r->w)) { r->ok = 0; return NULL; }
    r->ok = 1;
    return r;
}

static void chart(const patch_t *pt, double u, double v, geo_t *g, double *K)
{
    long double Kl[ORC_MAXND], Ku[ORC_MAXND], Kv[ORC_MAXND];
    koorn_ld(pt->d, u, v, Kl, Ku, Kv);
    for (int c = 0; c < 3; ++c) {
        long double s = 0, su = 0, sv = 0;
        for (int i = 0; i < pt->nd; ++i) {
            s += pt->coef[c][i] * Kl[i];
            su += pt->coef[c][i] * Ku[i];
            sv += pt->coef[c][i] * Kv[i];
        }
        g->X[c] = s; g->Xu[c] = su; g->Xv[c] = sv;
    }
    g->n[0] = g->Xu[1] * g->Xv[2] - g->Xu[2] * g->Xv[1];
    g->n[1] = g->Xu[2] * g->Xv[0] - g->Xu[0] * g->Xv[2];
    g->n[2] = g->Xu[0] * g->Xv[1] - g->Xu[1] * g->Xv[0];
    g->J = sqrtl(g->n[0] * g->n[0] + g->n[1] * g->n[1] + g->n[2] * g->n[2]);
    if (K) for (int i = 0; i < pt->nd; ++i) K[i] = (double)Kl[i];
}

static int setup_patch(const orc_problem *pb, int64_t j, patch_t *pt)
{
    int d = pb->degree[j];
    const orc_ref *r = get_ref(pb, d);
    if (!r) return -1;
    pt->d = d; pt->nd = r->nd; pt->ref = r;
    const double *x = pb->xyz + 3 * pb->node_ptr[j];
    for (int c = 0; c < 3; ++c)
        for (int a = 0; a < r->nd; ++a) {
            long double s = 0;
            for (int l = 0; l < r->nd; ++l) s += (long double)r->V[a * r->nd + l] * x[3 * l + c];
            pt->coef[c][a] = s;
        }
    double dj = INFINITY;
    for (int l = 0; l < r->nd; ++l) {
        geo_t g;
        chart(pt, r->uv[2 * l], r->uv[2 * l + 1], &g, NULL);
        double q = sqrt((double)g.J * fabs(r->w[l]));
        if (q < dj) dj = q;
    }
    pt->dj = dj;
    double rho = 0.0;
    for (int l = 0; l < r->nd; ++l) {
        const double nx = sqrt(x[3 * l] * x[3 * l] + x[3 * l + 1] * x[3 * l + 1] + x[3 * l + 2] * x[3 * l + 2]);
        if (nx > rho) rho = nx;
    }
    pt->rho = rho;
    return 0;
}

/* Kernel times area element at source y = X(u,v) for target x
 * (Sections 1 and 3):
 *   alpha G_k(r) J + beta n.(x-y) (1 - i k r) e^{ikr} / (4 pi r^3),
 * n = X_u x X_v unnormalised (it carries J).  The separation and n.(x-y)
 * are formed in long double. */
static cplx kernel_val(const kern_t *kk, const long double x[3], const geo_t *g)
{
    long double dl[3] = {x[0] - g->X[0], x[1] - g->X[1], x[2] - g->X[2]};
    double r = (double)sqrtl(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
    double nd = (double)(g->n[0] * dl[0] + g->n[1] * dl[1] + g->n[2] * dl[2]);
    double J = (double)g->J;
    cplx e = cexp(IU * kk->k * r);
    cplx G = e / (4.0 * ORC_PI * r);
    cplx D = nd * (1.0 - IU * kk->k * r) * e / (4.0 * ORC_PI * r * r * r);
    return kk->alpha * G * J + kk->beta * D;
}

/* Moments of the kernel against K_nm with a rule on triangle T given by
 * vertices (in T0 coordinates); weights scaled by |T|/|T0|. */
static void tri_moments(const patch_t *pt, const kern_t *kk, const long double x[3],
                        const double tri[6], const double *rule, int nq, cplx *mom, double *noise2)
{
    double ax = tri[0], ay = tri[1];
    double e1x = tri[2] - ax, e1y = tri[3] - ay, e2x = tri[4] - ax, e2y = tri[5] - ay;
    double scale = fabs(e1x * e2y - e1y * e2x); /* = |T| / |T0| */
    for (int i = 0; i < pt->nd; ++i) mom[i] = 0;
    double K[ORC_MAXND];
    const double bmag = cabs(kk->beta);
    double g2 = 0.0;
    for (int q = 0; q < nq; ++q) {
        double u = ax + rule[3 * q] * e1x + rule[3 * q + 1] * e2x;
        double v = ay + rule[3 * q] * e1y + rule[3 * q + 1] * e2y;
        geo_t g;
        chart(pt, u, v, &g, K);
        const double w = rule[3 * q + 2] * scale;
        cplx f = kernel_val(kk, x, &g) * w;
        double kk2 = 0.0;
        for (int i = 0; i < pt->nd; ++i) {
            mom[i] += f * K[i];
            kk2 += K[i] * K[i];
        }
        /* sensitivity of this node's contribution to the separation
         * x - X (whose rounding error scales with the coordinates): the
         * single layer moves by ~|f|/r and the double layer's numerator
         * n.(x - X) by ~b = |beta| J w / (4 pi r^3) per unit length;
         * (|f|^2 / r^2 + b^2) |K|^2 */
        const long double dl[3] = {x[0] - g.X[0], x[1] - g.X[1], x[2] - g.X[2]};
        const double r2 = (double)(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
        const double b = bmag * (double)g.J * w / (4.0 * ORC_PI * r2 * sqrt(r2));
        const double fa2 = creal(f) * creal(f) + cimag(f) * cimag(f);
        g2 += (fa2 / r2 + b * b) * kk2;
    }
    if (noise2) *noise2 = g2;
}

static double cnorm_diff(int nd, const cplx *a, const cplx *b)
{
    double s = 0;
    for (int i = 0; i < nd; ++i) {
        cplx t = a[i] - b[i];
        s += creal(t) * creal(t) + cimag(t) * cimag(t);
    }
    return sqrt(s);
}

static double cnorm(int nd, const cplx *a)
{
    double s = 0;
    for (int i = 0; i < nd; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return sqrt(s);
}

/* Adaptive near quadrature of Section 4.3 for one (target, patch) pair.
 * Depth-first over the 1->4 midpoint quadtree of T0. */
typedef struct {
    double tri[6];
    int depth;
    uint64_t code;   /* path in the quadtree: child indices in base 4 */
    cplx I[ORC_MAXND];
} node_t;

/* optional trace of the checked triangles ((depth << 56) | code), for tests
 * that study the shape of the subdivision trees */
static uint64_t *g_trace = NULL;
static int64_t g_trace_cap = 0, g_trace_n = 0;

void orc_set_trace(uint64_t *buf, int64_t cap)
{
    g_trace = buf;
    g_trace_cap = cap;
    g_trace_n = 0;
}

int64_t orc_trace_count(void) { return g_trace_n; }

static int near_moments(const patch_t *pt, const kern_t *kk, const long double x[3], double tau,
                        const double *rule, int nq, int max_depth, int truth, cplx *tot,
                        orc_stats *st)
{
    int nd = pt->nd;
    int cap = 1024;
    node_t *stk = malloc(sizeof(node_t) * cap);
    int sp = 0;
    node_t root = {{0, 0, 1, 0, 0, 1}, 0, 0, {0}};
    tri_moments(pt, kk, x, root.tri, rule, nq, root.I, NULL);
    st->visits += 1;
    stk[sp++] = root;
    for (int i = 0; i < nd; ++i) tot[i] = 0;
    int nonconv = 0;
    while (sp > 0) {
        node_t T = stk[--sp];
        if (g_trace && g_trace_n < g_trace_cap)
            g_trace[g_trace_n++] = ((uint64_t)T.depth << 56) | T.code;
        double a[2] = {T.tri[0], T.tri[1]}, b[2] = {T.tri[2], T.tri[3]}, c[2] = {T.tri[4], T.tri[5]};
        double ab[2] = {0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1])};
        double bc[2] = {0.5 * (b[0] + c[0]), 0.5 * (b[1] + c[1])};
        double ca[2] = {0.5 * (c[0] + a[0]), 0.5 * (c[1] + a[1])};
        node_t ch[4];
        double tris[4][6] = {
            {a[0], a[1], ab[0], ab[1], ca[0], ca[1]},
            {ab[0], ab[1], b[0], b[1], bc[0], bc[1]},
            {ca[0], ca[1], bc[0], bc[1], c[0], c[1]},
            {bc[0], bc[1], ca[0], ca[1], ab[0], ab[1]}};
        cplx S[ORC_MAXND];
        for (int i = 0; i < nd; ++i) S[i] = 0;
        double noise2 = 0.0;
        for (int k = 0; k < 4; ++k) {
            memcpy(ch[k].tri, tris[k], sizeof(tris[k]));
            ch[k].depth = T.depth + 1;
            ch[k].code = T.code * 4 + (uint64_t)k;
            double n2;
            tri_moments(pt, kk, x, ch[k].tri, rule, nq, ch[k].I, &n2);
            noise2 += n2;
            for (int i = 0; i < nd; ++i) S[i] += ch[k].I[i];
        }
        st->visits += 4;
        st->checks += 1;
        double area = ldexp(1.0, -2 * T.depth);  /* |T| / |T0| */
        double err = cnorm_diff(nd, S, T.I);
        double thr = tau * area;
        if (truth) {
            /* the integrand carries relative noise ~1e-15 |X| / r from the
             * chart evaluation; a per-triangle relative guard of 2e-12 keeps
             * the test above that floor (truth accuracy ~1e-12 relative) */
            double g = 2e-12 * cnorm(nd, S);
            if (g > thr) thr = g;
        }
        int accept = err <= thr;
        if (!truth) {
            /* rounding floor: the difference is accepted at the estimated
             * double-precision rounding level of the moments, which the
             * scaled threshold of deep subtriangles near a target can fall
             * below: u (|x| + rho_j) times the children's sensitivities,
             * doubled for the parent's and for the squared bound */
            const double u = 0x1p-53;
            const double sc = (double)sqrtl(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) + pt->rho;
            if (err <= ORC_NOISE_KAPPA * u * sc * 2.0 * sqrt(noise2)) accept = 1;
        }
        if (!accept && T.depth + 1 >= max_depth) { accept = 1; nonconv = 1; }
        if (accept) {
            for (int i = 0; i < nd; ++i) tot[i] += S[i];
            if (T.depth + 1 > st->max_level) st->max_level = T.depth + 1;
        } else {
            if (sp + 4 > cap) { cap *= 2; stk = realloc(stk, sizeof(node_t) * cap); }
            for (int k = 3; k >= 0; --k) stk[sp++] = ch[k];
        }
    }
    free(stk);
    if (nonconv) st->nonconverged += 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* 1-D adaptive Gauss-Legendre for vector (nd complex) integrands.     */
/* ------------------------------------------------------------------ */
typedef void (*vfun_t)(double t, void *ctx, cplx *out);

static double g_gl20x[20], g_gl20w[20];
static int g_gl20_ok = 0;

static void gl20_init(void)
{
    if (!g_gl20_ok) {
        orc_gauss_jacobi(20, 0, 0, g_gl20x, g_gl20w);
        g_gl20_ok = 1;
    }
}

static void gl_interval(vfun_t f, void *ctx, double a, double b, int nd, cplx *out)
{
    cplx tmp[ORC_MAXND];
    for (int i = 0; i < nd; ++i) out[i] = 0;
    for (int q = 0; q < 20; ++q) {
        f(a + (b - a) * g_gl20x[q], ctx, tmp);
        double w = (b - a) * g_gl20w[q];
        for (int i = 0; i < nd; ++i) out[i] += w * tmp[i];
    }
}

typedef struct { double a, b; double err; cplx I[ORC_MAXND]; } seg_t;

/* Estimate on [a,b]: the sum of Gauss-Legendre on the two halves; its error
 * estimate is the distance to Gauss-Legendre on the whole interval. */
static void seg_eval(vfun_t f, void *ctx, double a, double b, int nd, const cplx *whole,
                     seg_t *s, int64_t *nevals)
{
    cplx L[ORC_MAXND], R[ORC_MAXND];
    double m = 0.5 * (a + b);
    gl_interval(f, ctx, a, m, nd, L);
    gl_interval(f, ctx, m, b, nd, R);
    *nevals += 40;
    s->a = a; s->b = b;
    for (int i = 0; i < nd; ++i) s->I[i] = L[i] + R[i];
    s->err = cnorm_diff(nd, s->I, whole);
}

/* Globally adaptive 1-D integration (in the spirit of QUADPACK's QAG):
 * keep a list of intervals with estimates and error estimates; split the
 * interval with the largest error until the summed error is at most
 * max(tol (b - a), rel_guard ||sum||) or max_iv intervals are in use.  The
 * relative guard stops the refinement at the rounding floor of the
 * integrand; the interval budget bounds the cost (next to the self target
 * the double-layer numerator n(y).(x - X(y)) = O(s^2) is formed from O(s)
 * factors and carries relative noise ~1e-19 / s^2). */
static void adapt1d(vfun_t f, void *ctx, double a, double b, double tol, double rel_guard,
                    int max_iv, int nd, cplx *out, int64_t *nevals)
{
    seg_t *iv = malloc(sizeof(seg_t) * max_iv);
    cplx whole[ORC_MAXND];
    gl_interval(f, ctx, a, b, nd, whole);
    *nevals += 20;
    seg_eval(f, ctx, a, b, nd, whole, &iv[0], nevals);
    int n = 1;
    for (;;) {
        cplx S[ORC_MAXND];
        double E = 0.0;
        int worst = 0;
        for (int i = 0; i < nd; ++i) S[i] = 0;
        for (int k = 0; k < n; ++k) {
            for (int i = 0; i < nd; ++i) S[i] += iv[k].I[i];
            E += iv[k].err;
            if (iv[k].err > iv[worst].err) worst = k;
        }
        double thr = tol * (b - a), g = rel_guard * cnorm(nd, S);
        if (g > thr) thr = g;
        if (E <= thr || n + 1 > max_iv) {
            for (int i = 0; i < nd; ++i) out[i] = S[i];
            break;
        }
        /* intervals below 1e-7 of the range are accepted as they are: their
         * share of the integral is below the tolerances checked, while the
         * integrand's rounding noise grows as they shrink towards the
         * singular point */
        if (iv[worst].b - iv[worst].a < 1e-7 * (b - a)) {
            iv[worst].err = 0.0;
            continue;
        }
        /* split the worst interval: its two halves become intervals */
        seg_t w = iv[worst];
        double m = 0.5 * (w.a + w.b);
        cplx hl[ORC_MAXND], hr[ORC_MAXND];
        gl_interval(f, ctx, w.a, m, nd, hl);
        gl_interval(f, ctx, m, w.b, nd, hr);
        *nevals += 40;
        seg_eval(f, ctx, w.a, m, nd, hl, &iv[worst], nevals);
        seg_eval(f, ctx, m, w.b, nd, hr, &iv[n], nevals);
        ++n;
    }
    free(iv);
}

/* Self quadrature: target at reference node t = (ut, vt) of its own
 * patch.  T0 = union of the triangles (t, P_i, P_{i+1}); each is mapped
 * by y = t + s (P_i + lam (P_{i+1} - P_i) - t), s, lam in [0,1], with
 * area element s * |det(P_i - t, P_{i+1} - P_i)| ds dlam, which removes
 * the 1/r singularity.  Nested adaptive Gauss-Legendre in s and lam. */
typedef struct {
    const patch_t *pt;
    const kern_t *kk;
    long double x[3];
    qreal xq[3];
    double t[2], P0[2], P1[2], det;
    double lam;
    double tol_in;
    int64_t *nevals;
} self_ctx;

/* Quad-precision (__float128) chart position and normal for the self
 * integrand: next to the target the double-layer numerator
 * n(y).(X(t) - X(y)) = O(s^2) is formed from O(s) factors; in quad precision
 * its rounding noise (~1e-34 / s^2) stays far below every tolerance the
 * adaptive tests use. */
static qreal ipowq_(qreal x, int e)
{
    if (e < 0) return 0;
    qreal r = 1;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

static void koorn_q(int d, qreal u, qreal v, qreal *K, qreal *Ku, qreal *Kv)
{
    for (int n = 0; n <= d; ++n)
        for (int m = 0; m <= n; ++m) {
            int k = n - m, b = 2 * m + 1;
            qreal A = 0, Av = 0;
            for (int s = 0; s <= k; ++s) {
                qreal c = (qreal)binom(k, k - s) * (qreal)binom(k + b, s);
                A += c * ipowq_(-v, s) * ipowq_(1 - v, k - s);
                Av += c * (-(qreal)s * ipowq_(-v, s - 1) * ipowq_(1 - v, k - s)
                           - (qreal)(k - s) * ipowq_(-v, s) * ipowq_(1 - v, k - s - 1));
            }
            qreal B = 0, Bu = 0, Bv = 0, w = u + v - 1;
            for (int s = 0; s <= m; ++s) {
                qreal c = (qreal)binom(m, s) * (qreal)binom(m, s);
                B += c * ipowq_(w, s) * ipowq_(u, m - s);
                Bu += c * ((qreal)s * ipowq_(w, s - 1) * ipowq_(u, m - s)
                           + (qreal)(m - s) * ipowq_(w, s) * ipowq_(u, m - s - 1));
                Bv += c * (qreal)s * ipowq_(w, s - 1) * ipowq_(u, m - s);
            }
            /* c_nm = sqrt(2(n+1)(2m+1)) to quad precision: long double
             * square root refined by one Newton step */
            qreal c2 = (qreal)(2 * (n + 1) * (2 * m + 1));
            qreal cn = (qreal)sqrtl((long double)c2);
            cn = 0.5 * (cn + c2 / cn);
            int idx = n * (n + 1) / 2 + m;
            K[idx] = cn * A * B;
            Ku[idx] = cn * A * Bu;
            Kv[idx] = cn * (Av * B + A * Bv);
        }
}

/* X(u,v) and n = X_u x X_v in quad precision, u = ut + s*du etc. formed in
 * quad precision as well. */
static void chart_q(const patch_t *pt, qreal u, qreal v, qreal X[3], qreal n[3])
{
    qreal K[ORC_MAXND], Ku[ORC_MAXND], Kv[ORC_MAXND], Xu[3], Xv[3];
    koorn_q(pt->d, u, v, K, Ku, Kv);
    for (int c = 0; c < 3; ++c) {
        qreal a = 0, au = 0, av = 0;
        for (int i = 0; i < pt->nd; ++i) {
            qreal cf = (qreal)pt->coef[c][i];
            a += cf * K[i];
            au += cf * Ku[i];
            av += cf * Kv[i];
        }
        X[c] = a; Xu[c] = au; Xv[c] = av;
    }
    n[0] = Xu[1] * Xv[2] - Xu[2] * Xv[1];
    n[1] = Xu[2] * Xv[0] - Xu[0] * Xv[2];
    n[2] = Xu[0] * Xv[1] - Xu[1] * Xv[0];
}

static void self_inner(double s, void *vctx, cplx *out)
{
    self_ctx *c = (self_ctx *)vctx;
    const patch_t *pt = c->pt;
    qreal ex = (qreal)c->P0[0] + (qreal)c->lam * ((qreal)c->P1[0] - c->P0[0]) - c->t[0];
    qreal ey = (qreal)c->P0[1] + (qreal)c->lam * ((qreal)c->P1[1] - c->P0[1]) - c->t[1];
    qreal uq = (qreal)c->t[0] + (qreal)s * ex, vq = (qreal)c->t[1] + (qreal)s * ey;
    qreal X[3], n[3];
    chart_q(pt, uq, vq, X, n);
    qreal dl[3] = {c->xq[0] - X[0], c->xq[1] - X[1], c->xq[2] - X[2]};
    double r = (double)sqrtl((long double)(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]));
    double ndx = (double)(n[0] * dl[0] + n[1] * dl[1] + n[2] * dl[2]);
    double J = (double)sqrtl((long double)(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]));
    const kern_t *kk = c->kk;
    cplx e = cexp(IU * kk->k * r);
    cplx G = e / (4.0 * ORC_PI * r);
    cplx D = ndx * (1.0 - IU * kk->k * r) * e / (4.0 * ORC_PI * r * r * r);
    cplx f = (kk->alpha * G * J + kk->beta * D) * s * c->det;
    double K[ORC_MAXND];
    orc_koornwinder(pt->d, (double)uq, (double)vq, K, NULL, NULL);
    for (int i = 0; i < pt->nd; ++i) out[i] = f * K[i];
}

static void self_outer(double lam, void *vctx, cplx *out)
{
    self_ctx *c = (self_ctx *)vctx;
    c->lam = lam;
    adapt1d(self_inner, c, 0.0, 1.0, c->tol_in, 1e-12, 60, c->pt->nd, out, c->nevals);
}

/* The self target is the chart point X(u_t, v_t) itself (it equals the
 * input node to interpolation rounding); taking the input node instead would
 * put a spurious near-singularity ~1e-16 off the surface. */
static void self_moments(const patch_t *pt, const kern_t *kk, double ut, double vt, double tau,
                         cplx *tot, orc_stats *st)
{
    gl20_init();
    geo_t gt;
    chart(pt, ut, vt, &gt, NULL);
    const long double *x = gt.X;
    double V[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    int nd = pt->nd;
    for (int i = 0; i < nd; ++i) tot[i] = 0;
    for (int e = 0; e < 3; ++e) {
        self_ctx c;
        c.pt = pt; c.kk = kk;
        for (int q = 0; q < 3; ++q) c.x[q] = x[q];
        {
            qreal Xq[3], nq[3];
            chart_q(pt, (qreal)ut, (qreal)vt, Xq, nq);
            for (int q = 0; q < 3; ++q) c.xq[q] = Xq[q];
        }
        c.t[0] = ut; c.t[1] = vt;
        c.P0[0] = V[e][0]; c.P0[1] = V[e][1];
        c.P1[0] = V[(e + 1) % 3][0]; c.P1[1] = V[(e + 1) % 3][1];
        double ax = c.P0[0] - ut, ay = c.P0[1] - vt;
        double bx = c.P1[0] - c.P0[0], by = c.P1[1] - c.P0[1];
        c.det = fabs(ax * by - ay * bx);
        c.tol_in = tau / 3.0 * 0.1;
        c.nevals = &st->self_evals;
        cplx part[ORC_MAXND];
        /* the outer integrand inherits the inner accuracy as noise */
        adapt1d(self_outer, &c, 0.0, 1.0, tau / 3.0, 1e-11, 80, nd, part, &st->self_evals);
        for (int i = 0; i < nd; ++i) tot[i] += part[i];
    }
    st->self_targets += 1;
}

/* ------------------------------------------------------------------ */
/* Public entry points                                                  */
/* ------------------------------------------------------------------ */
static kern_t make_kernel(const orc_problem *pb)
{
    kern_t kk;
    kk.alpha = pb->alpha_re + IU * pb->alpha_im;
    kk.beta = pb->beta_re + IU * pb->beta_im;
    kk.k = pb->k_re + IU * pb->k_im;
    return kk;
}

static int64_t patch_of_node(const orc_problem *pb, int64_t node)
{
    int64_t lo = 0, hi = pb->P - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (pb->node_ptr[mid] <= node) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Weights a^j_l(x_t), l = 0..nd-1, of one pair (target t, patch j); a self
 * pair when j is the patch of target t's node.  out: interleaved complex. */
int orc_pair_weights(const orc_problem *pb, int64_t t, int64_t j, double *out, orc_stats *st)
{
    patch_t pt;
    if (setup_patch(pb, j, &pt)) return -1;
    kern_t kk = make_kernel(pb);
    long double x[3] = {pb->txyz[3 * t], pb->txyz[3 * t + 1], pb->txyz[3 * t + 2]};
    int nd = pt.nd;
    cplx Imom[ORC_MAXND];
    int truth = pb->mode == 1;
    /* truth mode: 1e-12 in the same scaled norm (far below any tolerance
     * the method is run at) with a 1e-14 relative guard per (sub)interval
     * against the rounding floor */
    double tau = (truth ? 1e-12 : pb->loosen * pb->tol) * pt.dj / pt.ref->normV;
    int64_t node = pb->node_of_target[t];
    int is_self = node >= 0 && patch_of_node(pb, node) == j;
    if (is_self) {
        int64_t l = node - pb->node_ptr[j];
        self_moments(&pt, &kk, pt.ref->uv[2 * l], pt.ref->uv[2 * l + 1],
                     truth ? tau : 0.1 * tau, Imom, st);
    } else {
        /* method mode: 8 x 8 conical product (exact to degree 15) unless set */
        int ng = truth ? 20 : (pb->ng > 0 ? pb->ng : 8);
        double *rule = malloc(sizeof(double) * 3 * ng * ng);
        if (orc_conical_rule(ng, rule)) { free(rule); return -2; }
        near_moments(&pt, &kk, x, tau, rule, ng * ng, pb->max_depth, truth, Imom, st);
        st->near_pairs += 1;
        free(rule);
    }
    for (int l = 0; l < nd; ++l) {
        cplx s = 0;
        for (int a = 0; a < nd; ++a) s += pt.ref->V[a * nd + l] * Imom[a];
        out[2 * l] = creal(s);
        out[2 * l + 1] = cimag(s);
    }
    return 0;
}

/* CSR-by-target layout: row t holds, in ascending patch order, the blocks of
 * every patch of T_eta(x_t) and (for node targets) of the target's own
 * patch; inside a block the patch's nodes in order. */
int orc_row_ptr(const orc_problem *pb, int64_t *row_ptr)
{
    row_ptr[0] = 0;
    for (int64_t t = 0; t < pb->NT; ++t) {
        int64_t len = 0;
        for (int64_t e = pb->near_row_ptr[t]; e < pb->near_row_ptr[t + 1]; ++e)
            len += orc_nd(pb->degree[pb->near_patch[e]]);
        int64_t node = pb->node_of_target[t];
        if (node >= 0) len += orc_nd(pb->degree[patch_of_node(pb, node)]);
        row_ptr[t + 1] = row_ptr[t] + len;
    }
    return 0;
}

/* Fill col/val for targets [t0, t1) (val interleaved complex). */
int orc_generate_rows(const orc_problem *pb, int64_t t0, int64_t t1, const int64_t *row_ptr,
                      int32_t *col, double *val, orc_stats *st)
{
    double buf[2 * ORC_MAXND];
    for (int64_t t = t0; t < t1; ++t) {
        int64_t node = pb->node_of_target[t];
        int64_t own = node >= 0 ? patch_of_node(pb, node) : -1;
        int64_t pos = row_ptr[t];
        int64_t e = pb->near_row_ptr[t], e1 = pb->near_row_ptr[t + 1];
        int own_done = own < 0;
        while (e < e1 || !own_done) {
            int64_t j;
            if (!own_done && (e >= e1 || own < pb->near_patch[e])) { j = own; own_done = 1; }
            else { j = pb->near_patch[e++]; }
            int rc = orc_pair_weights(pb, t, j, buf, st);
            if (rc) return rc;
            int nd = orc_nd(pb->degree[j]);
            for (int l = 0; l < nd; ++l) {
                col[pos] = (int32_t)(pb->node_ptr[j] + l);
                val[2 * pos] = buf[2 * l];
                val[2 * pos + 1] = buf[2 * l + 1];
                ++pos;
            }
        }
        if (pos != row_ptr[t + 1]) return -3;
    }
    return 0;
}

/* y = A sigma (complex), the local-correction part of the apply step. */
int orc_apply(int64_t NT, const int64_t *row_ptr, const int32_t *col, const double *val,
              const double *sigma, double *y)
{
    for (int64_t t = 0; t < NT; ++t) {
        cplx s = 0;
        for (int64_t e = row_ptr[t]; e < row_ptr[t + 1]; ++e) {
            cplx a = val[2 * e] + IU * val[2 * e + 1];
            cplx g = sigma[2 * col[e]] + IU * sigma[2 * col[e] + 1];
            s += a * g;
        }
        y[2 * t] = creal(s);
        y[2 * t + 1] = cimag(s);
    }
    return 0;
}

/* Per-patch quantities exposed for tests: d_j and ||V||. */
int orc_patch_info(const orc_problem *pb, int64_t j, double *dj, double *normV)
{
    patch_t pt;
    if (setup_patch(pb, j, &pt)) return -1;
    *dj = pt.dj;
    *normV = pt.ref->normV;
    return 0;
}

/* Bounding ball of patch j for the near-field definitions of Section 4.
 * Centre: the parametric mean of the chart, (1/|T0|) int_T0 X du dv,
 * integrated with the conical rule of 8 x 8 points (exact for polynomials of
 * degree <= 15 >= d).  Radius: the largest |X(u,v) - c| over the lattice
 * (i/lat, k/lat), i + k <= lat, of T0, corners and edges included. */
int orc_patch_ball(const orc_problem *pb, int64_t j, int lat, double *c3, double *R)
{
    patch_t pt;
    if (setup_patch(pb, j, &pt)) return -1;
    double rule[64 * 3];
    if (orc_conical_rule(8, rule)) return -2;
    long double c[3] = {0, 0, 0}, area = 0;
    for (int q = 0; q < 64; ++q) {
        geo_t g;
        chart(&pt, rule[3 * q], rule[3 * q + 1], &g, NULL);
        for (int a = 0; a < 3; ++a) c[a] += rule[3 * q + 2] * g.X[a];
        area += rule[3 * q + 2];
    }
    for (int a = 0; a < 3; ++a) c3[a] = (double)(c[a] / area);
    double r2 = 0.0;
    for (int i = 0; i <= lat; ++i)
        for (int k = 0; i + k <= lat; ++k) {
            geo_t g;
            chart(&pt, (double)i / lat, (double)k / lat, &g, NULL);
            double s = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double d = (double)g.X[a] - c3[a];
                s += d * d;
            }
            if (s > r2) r2 = s;
        }
    *R = sqrt(r2);
    return 0;
}

/* Chart evaluation for tests: X, X_u, X_v of patch j at (u,v). */
int orc_chart(const orc_problem *pb, int64_t j, double u, double v, double *out9)
{
    patch_t pt;
    if (setup_patch(pb, j, &pt)) return -1;
    geo_t g;
    chart(&pt, u, v, &g, NULL);
    for (int c = 0; c < 3; ++c) {
        out9[c] = (double)g.X[c];
        out9[3 + c] = (double)g.Xu[c];
        out9[6 + c] = (double)g.Xv[c];
    }
    return 0;
}
