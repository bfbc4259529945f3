// device.hpp -- device-side building blocks shared by the quadrature kernels:
// chart evaluation through the Koornwinder recurrences, the layer-potential
// kernel (Sections 1 and 3 of the paper) and wavefront reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "fastmath.hpp"
#include "koorn.hpp"

namespace nfq {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;  // 1/(4 pi)

struct Kern {
    double ar, ai, br, bi, kr, ki;  // alpha, beta, wavenumber
    double bm;                      // |beta|
};

// Rounding floor of the adaptive test.  A node's moment contribution moves
// by about (|f|/r + b) |dX| when the separation x - X(y) is off by |dX|
// (b = |beta| J w / (4 pi r^3) for the double layer's numerator), and |dX|
// is a few units of roundoff times the coordinate scale |x| + max_l |x_l|.
// A test whose difference lies below kNoiseKappa times that level, summed
// in quadrature over the children's nodes (doubled for the parent and for
// the squared bound), is accepted: refining further cannot reduce it.
constexpr double kNoiseKappa = 16.0;
constexpr double kUnitRoundoff = 0x1p-53;

__device__ __forceinline__ double noise_factor(double scale)
{
    const double g = 2.0 * kNoiseKappa * kUnitRoundoff * scale;
    return g * g;
}

// Values of the Koornwinder basis at (u,v) into K[ND], and the chart
// X = sum_a coef[c*ND + a] K_a with its derivatives (Section 3.2).
template <int D>
__device__ __forceinline__ void chart_eval(const double *__restrict__ coef, double u, double v,
                                           double *K, double X[3], double Xu[3], double Xv[3])
{
    constexpr int ND = nd_of(D);
#pragma unroll
    for (int c = 0; c < 3; ++c) X[c] = Xu[c] = Xv[c] = 0.0;
    koorn_visit<D>(u, v, [&](int a, double k, double ku, double kv) {
        K[a] = k;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double cf = coef[c * ND + a];
            X[c] = __builtin_fma(cf, k, X[c]);
            Xu[c] = __builtin_fma(cf, ku, Xu[c]);
            Xv[c] = __builtin_fma(cf, kv, Xv[c]);
        }
    });
}

// Kernel value times area element at source y with unnormalised normal n
// (|n| = J) for target x:
//   alpha G_k(r) J + beta n.(x-y) (1 - i k r) e^{ikr} / (4 pi r^3).
// Returns (re, im).  `helm` selects the Helmholtz path (k != 0).
__device__ __forceinline__ void kern_eval(const Kern &k, bool helm, const double x[3],
                                          const double y[3], const double n[3], double &fr,
                                          double &fi, int &singular, double &sens)
{
    const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) singular = 1;
    const double rinv = rsqrt_nr(r2);
    const double J = __builtin_sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double nd = n[0] * dx + n[1] * dy + n[2] * dz;
    const double g0 = kInv4Pi * rinv;            // 1/(4 pi r)
    const double d0 = g0 * nd * rinv * rinv;     // n.(x-y)/(4 pi r^3)
    const double rinv2 = rinv * rinv;
    const double bsens = k.bm * g0 * J * rinv2;  // |beta| J / (4 pi r^3)
    if (!helm) {
        // e^{ikr} = 1, (1 - ikr) = 1
        fr = k.ar * g0 * J + k.br * d0;
        fi = k.ai * g0 * J + k.bi * d0;
        sens = (fr * fr + fi * fi) * rinv2 + bsens * bsens;
        return;
    }
    const double r = r2 * rinv;
    double s, c;
    sincos_cw(k.kr * r, &s, &c);
    if (k.ki != 0.0) {
        const double damp = exp(-k.ki * r);
        s *= damp;
        c *= damp;
    }
    // (1 - i k r) with complex k: (1 + ki r) - i kr r
    const double pr = 1.0 + k.ki * r, pi = -k.kr * r;
    // G J = g0 J e ; D = d0 (1 - ikr) e
    const double gr = g0 * J * c, gi = g0 * J * s;
    const double qr = d0 * (pr * c - pi * s), qi = d0 * (pr * s + pi * c);
    fr = k.ar * gr - k.ai * gi + k.br * qr - k.bi * qi;
    fi = k.ar * gi + k.ai * gr + k.br * qi + k.bi * qr;
    sens = (fr * fr + fi * fi) * rinv2 + bsens * bsens;
}

__device__ __forceinline__ void kern_eval(const Kern &k, bool helm, const double x[3],
                                          const double y[3], const double n[3], double &fr,
                                          double &fi, int &singular)
{
    double sens;
    kern_eval(k, helm, x, y, n, fr, fi, singular, sens);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_or(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v |= __shfl_xor(v, off, 64);
    return v;
}

}  // namespace nfq
