// koorn.hpp -- Koornwinder basis on T0 by three-term recurrences, for host
// and device (Section 2 of the paper: K_nm(u,v) = c_nm (1-v)^m
// P^{(0,2m+1)}_{n-m}(1-2v) P_m((2u+v-1)/(1-v)), orthonormal on T0 with
// c_nm = sqrt(2 (n+1) (2m+1)); index of (n,m) is n(n+1)/2 + m).
//
// The Legendre factor is carried in homogeneous form B_m = (1-v)^m P_m(xi),
// which obeys (m+1) B_{m+1} = (2m+1) s B_m - m q B_{m-1}, s = 2u+v-1,
// q = (1-v)^2 (no division by 1-v).  The Jacobi factor A_k = P^{(0,b)}_k(x),
// x = 1 - 2v, b = 2m+1, follows the standard Jacobi three-term recurrence.
// Derivatives are carried through both recurrences.
#pragma once

#ifndef NFQ_HD
#if defined(__HIPCC__)
#define NFQ_HD __host__ __device__
#else
#define NFQ_HD
#endif
#endif

namespace nfq {

NFQ_HD constexpr int nd_of(int d) { return (d + 1) * (d + 2) / 2; }

// Visit every (n, m, K, dK/du, dK/dv) for n <= D.  F is called as
// f(idx, K, Ku, Kv).
template <int D, typename F>
NFQ_HD inline void koorn_visit(double u, double v, F &&f)
{
    const double s = 2.0 * u + v - 1.0;
    const double om = 1.0 - v;
    const double q = om * om;
    const double x = 1.0 - 2.0 * v;
    double Bm1 = 0.0, Bm1u = 0.0, Bm1v = 0.0;  // B_{m-1}
    double Bm = 1.0, Bmu = 0.0, Bmv = 0.0;      // B_m
#pragma unroll
    for (int m = 0; m <= D; ++m) {
        const double b = 2.0 * m + 1.0;
        // Jacobi P^{(0,b)}_k(x) and d/dv, k = 0..D-m
        double Ak1 = 0.0, Ak1v = 0.0;  // A_{k-1}
        double Ak = 1.0, Akv = 0.0;    // A_k
#pragma unroll
        for (int k = 0; k <= D - m; ++k) {
            const int n = m + k;
            const double c = __builtin_sqrt(2.0 * (n + 1) * (2 * m + 1));
            const int idx = n * (n + 1) / 2 + m;
            f(idx, c * Ak * Bm, c * Ak * Bmu, c * (Akv * Bm + Ak * Bmv));
            if (k < D - m) {
                // 2(k+1)(k+b+1)(2k+b) A_{k+1} =
                //   (2k+b+1)[(2k+b+2)(2k+b) x - b^2] A_k - 2k(k+b)(2k+b+2) A_{k-1}
                const double kk = (double)k;
                const double den = 2.0 * (kk + 1.0) * (kk + b + 1.0) * (2.0 * kk + b);
                const double ca = (2.0 * kk + b + 1.0) * (2.0 * kk + b + 2.0) * (2.0 * kk + b) / den;
                const double cb = -(2.0 * kk + b + 1.0) * b * b / den;
                const double cc = 2.0 * kk * (kk + b) * (2.0 * kk + b + 2.0) / den;
                const double An = (ca * x + cb) * Ak - cc * Ak1;
                // dx/dv = -2
                const double Anv = -2.0 * ca * Ak + (ca * x + cb) * Akv - cc * Ak1v;
                Ak1 = Ak; Ak1v = Akv;
                Ak = An; Akv = Anv;
            }
        }
        if (m < D) {
            const double mm = (double)m;
            // (m+1) B_{m+1} = (2m+1) s B_m - m q B_{m-1}; ds/du = 2, ds/dv = 1,
            // dq/du = 0, dq/dv = -2(1-v)
            const double inv = 1.0 / (mm + 1.0);
            const double Bn = ((2.0 * mm + 1.0) * s * Bm - mm * q * Bm1) * inv;
            const double Bnu = ((2.0 * mm + 1.0) * (2.0 * Bm + s * Bmu) - mm * q * Bm1u) * inv;
            const double Bnv = ((2.0 * mm + 1.0) * (Bm + s * Bmv)
                                - mm * (-2.0 * om * Bm1 + q * Bm1v)) * inv;
            Bm1 = Bm; Bm1u = Bmu; Bm1v = Bmv;
            Bm = Bn; Bmu = Bnu; Bmv = Bnv;
        }
    }
}

// Runtime-degree variant for host set-up code.
template <typename F>
inline void koorn_visit_rt(int d, double u, double v, F &&f)
{
    switch (d) {
    case 0: koorn_visit<0>(u, v, f); break;
    case 1: koorn_visit<1>(u, v, f); break;
    case 2: koorn_visit<2>(u, v, f); break;
    case 3: koorn_visit<3>(u, v, f); break;
    case 4: koorn_visit<4>(u, v, f); break;
    case 5: koorn_visit<5>(u, v, f); break;
    case 6: koorn_visit<6>(u, v, f); break;
    case 7: koorn_visit<7>(u, v, f); break;
    case 8: koorn_visit<8>(u, v, f); break;
    default: break;
    }
}

}  // namespace nfq
