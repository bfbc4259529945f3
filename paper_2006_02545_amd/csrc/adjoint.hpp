// adjoint.hpp -- gradient of Phi = sum_t conj(lambda_t) (A sigma)_t with
// respect to the patch nodes, the wavenumber and the kernel weights alpha,
// beta, for the quadrature the forward generator computes (frozen
// subdivision: the adaptive decisions are recomputed with the forward's own
// arithmetic, then the quadrature sum over the accepted subtriangles is
// differentiated).
//
// With sigma^j(u,v) = sum_nm s_nm K_nm(u,v), s = V sigma_j (Section 4.2) the
// functional is a sum over pairs and accepted rule nodes q of
//     w_q conj(lambda_t) sigma^j(y_q) Kern(x_t, X(y_q), n(y_q)).
// For a node with r = x - X, R = |r|, E = e^{ikR},
//     Kern = alpha J G + beta (n.r) F,  G = E/(4 pi R),
//     F = (1 - ikR) E / (4 pi R^3),  F' = E (k^2 R^2 + 3ikR - 3) / (4 pi R^4),
//     dKern/dX = -alpha J G' r/R - beta [F n + (n.r) F' r/R],
//     G' = E (ikR - 1) / (4 pi R^2),
//     dKern/dn = alpha G n/J + beta F r,
//     dKern/dk = alpha J iR G + beta (n.r) k E / (4 pi R),
// and dKern/dx_t = -dKern/dX.  The chart X = sum_nm chi_nm K_nm (chi = V x)
// gives, per node, dPhi/dchi_nm = gX K_nm + (X_v x gn) dK_nm/du
// + (gn x X_u) dK_nm/dv (gX, gn the weighted kernel derivatives), and
// dPhi/dx_l = sum_nm V_(nm),l dPhi/dchi_nm.
#pragma once

#include "near_patch.hpp"

namespace nfq {

// Per-node gradient terms.  Inputs: target x, chart X, Xu, Xv, weight wq
// (rule weight times |T|/|T0|), rho = conj(lambda) sigma(y) (complex).
// Outputs: gX, gn (complex 3-vectors, already times rho wq), gk, the single-
// and double-layer integrands phiS = J G rho wq, phiD = (n.r) F rho wq.
struct NodeGrad {
    double gXr[3], gXi[3], gnr[3], gni[3];
    double gkr, gki, sr, si, dr, di;
};

__device__ __forceinline__ void cmul(double ar, double ai, double br, double bi, double &cr,
                                     double &ci)
{
    cr = ar * br - ai * bi;
    ci = ar * bi + ai * br;
}

__device__ __forceinline__ void node_grad(const Kern &k, const double x[3], const double X[3],
                                          const double n[3], double wq, double rhor, double rhoi,
                                          NodeGrad &g)
{
    const double rx = x[0] - X[0], ry = x[1] - X[1], rz = x[2] - X[2];
    const double R2 = rx * rx + ry * ry + rz * rz;
    const double Rinv = rsqrt_nr(R2);
    const double R = R2 * Rinv;
    const double J = __builtin_sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double nr = n[0] * rx + n[1] * ry + n[2] * rz;
    double s, c;
    sincos_cw(k.kr * R, &s, &c);
    if (k.ki != 0.0) {
        const double damp = exp(-k.ki * R);
        s *= damp;
        c *= damp;
    }
    // E = c + i s;  k = kr + i ki;  kR = (kr R, ki R)
    const double q = kInv4Pi * Rinv;                 // 1/(4 pi R)
    const double Gr = c * q, Gi = s * q;             // G
    // ikR = (-ki R, kr R)
    const double ikRr = -k.ki * R, ikRi = k.kr * R;
    // F = (1 - ikR) E q / R^2
    double Fr, Fi;
    cmul(1.0 - ikRr, -ikRi, Gr, Gi, Fr, Fi);
    Fr *= Rinv * Rinv;
    Fi *= Rinv * Rinv;
    // G' = E (ikR - 1) q / R
    double Gpr, Gpi;
    cmul(ikRr - 1.0, ikRi, Gr, Gi, Gpr, Gpi);
    Gpr *= Rinv;
    Gpi *= Rinv;
    // F' = E (k^2 R^2 + 3 ikR - 3) q / R^3 ; k^2 R^2 = (kR)^2
    const double kRr = k.kr * R, kRi = k.ki * R;
    const double k2r = kRr * kRr - kRi * kRi, k2i = 2.0 * kRr * kRi;
    double Fpr, Fpi;
    cmul(k2r + 3.0 * ikRr - 3.0, k2i + 3.0 * ikRi, Gr, Gi, Fpr, Fpi);
    const double R3inv = Rinv * Rinv * Rinv;
    Fpr *= R3inv;
    Fpi *= R3inv;
    // weights: W = rho wq
    const double Wr = rhor * wq, Wi = rhoi * wq;
    // alpha W, beta W
    double aWr, aWi, bWr, bWi;
    cmul(k.ar, k.ai, Wr, Wi, aWr, aWi);
    cmul(k.br, k.bi, Wr, Wi, bWr, bWi);
    // dKern/dX = -alpha J G' r/R - beta [F n + (n.r) F' r/R]
    double t1r, t1i, t2r, t2i, t3r, t3i;
    cmul(aWr, aWi, Gpr, Gpi, t1r, t1i);            // alpha W G'
    t1r *= -J * Rinv;
    t1i *= -J * Rinv;
    cmul(bWr, bWi, Fr, Fi, t2r, t2i);              // beta W F
    cmul(bWr, bWi, Fpr, Fpi, t3r, t3i);            // beta W F'
    t3r *= -nr * Rinv;
    t3i *= -nr * Rinv;
    const double rv[3] = {rx, ry, rz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.gXr[a] = (t1r + t3r) * rv[a] - t2r * n[a];
        g.gXi[a] = (t1i + t3i) * rv[a] - t2i * n[a];
    }
    // dKern/dn = alpha G n/J + beta F r
    double u1r, u1i;
    cmul(aWr, aWi, Gr, Gi, u1r, u1i);
    const double Jinv = 1.0 / J;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.gnr[a] = u1r * n[a] * Jinv + t2r * rv[a];
        g.gni[a] = u1i * n[a] * Jinv + t2i * rv[a];
    }
    // dKern/dk = alpha J iR G + beta (n.r) k E q
    double v1r, v1i, v2r, v2i;
    cmul(u1r, u1i, 0.0, R * J, v1r, v1i);          // alpha W G * iR J
    double kEr, kEi;
    cmul(k.kr, k.ki, Gr, Gi, kEr, kEi);            // k E q
    cmul(bWr, bWi, kEr * nr, kEi * nr, v2r, v2i);
    g.gkr = v1r + v2r;
    g.gki = v1i + v2i;
    // single and double layer integrands (for dPhi/dalpha, dPhi/dbeta)
    cmul(Wr, Wi, Gr * J, Gi * J, g.sr, g.si);
    cmul(Wr, Wi, Fr * nr, Fi * nr, g.dr, g.di);
}

struct AdjArgs {
    PatchArgs pa;             // forward arguments (val unused)
    QuadArgs qa;              // self-rule arguments
    const double *scoef;      // sigma coefficients per patch: [2 * node_ptr[j] + 2 a + {re,im}]
    const double *lam;        // lambda per target (complex)
    const int64_t *cptr;      // first chunk index of each patch
    const int64_t *pptr;      // first patch-major near pair of each patch
    double *gc_item;          // [chunks][6 ND_pad]: chart-coefficient gradient per work item
    double *t_pair;           // [pairs][12]: target gradient, dk, phiS, phiD per pair
    double *gc_self;          // [N][6 ND_max]: chart-coefficient gradient per self pair (by node)
    int gc_pitch;             // item row: 6 + 18 ND_max (scalars, nine moment vectors)
    int self_pitch;           // 6 ND_max
};

// sigma(y) = sum_a s_a K_a (complex)
template <int ND>
__device__ __forceinline__ void sigma_at(const double *sc, const double *K, double &sr, double &si)
{
    sr = 0.0;
    si = 0.0;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        sr = __builtin_fma(sc[2 * a], K[a], sr);
        si = __builtin_fma(sc[2 * a + 1], K[a], si);
    }
}

// Adjoint of the near quadrature, one work item (patch, <= 64 targets) per
// workgroup.  The forward's subdivision walk is replayed with its own
// arithmetic (same work split, same tests).  After the test of a group, the
// targets that accepted its children are differentiated with one thread per
// child node: the thread sums the weighted kernel derivatives gX, gn over
// those targets, and the group adds to nine moment vectors per wavefront,
//     M[gX_c], M[(X_v x gn)_c], M[(gn x X_u)_c],  M[f]_m = sum_q f(q) K_m(q),
// each reduced over the wavefront's 64 nodes like the forward's moments.
// The chart-coefficient gradient follows at the end from the differentiation
// matrices of the basis:  dPhi/dchi_c = M[gX_c] + Du M[b_c] + Dv M[d_c].
template <int D>
__global__ __launch_bounds__(256, (D <= 4 ? 2 : 1)) void k_adjoint_patch(AdjArgs aa)
{
    using S = PatchShape<D, true>;
    constexpr int ND = S::ND, W = S::W, PL = S::PL, G0 = S::G0, KS = S::KS, R = S::R;
    constexpr int GSA = (KS + 7 + 6) | 1;   // forward row + X_u, X_v
    const PatchArgs &a = aa.pa;
    __shared__ double s_geo[256 * GSA];
    __shared__ GroupEntry s_stack[kGroupStack];
    __shared__ double s_x[64][3];
    __shared__ double s_lam[64][2];
    __shared__ int32_t s_pair[64];
    __shared__ double s_t[64][6];
    __shared__ double s_tw[2][4][6];
    __shared__ double s_sc[2 * KS];
    __shared__ double s_cf[3 * ND];
    __shared__ double s_cm[4 * W];
    __shared__ double s_g2[4];
    __shared__ double s_nf[64];
    // failing-target masks of the current and the next group (alternating)
    __shared__ unsigned long long s_fail2[2];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int grp16 = lane >> 4, l16 = lane & 15;
    double *mom = a.mom + (int64_t)blockIdx.x * a.mom_slot;
    auto mptr = [&](int L, int c, int s) { return mom + ((int64_t)(L * 4 + c) * 64 + s) * W; };
    int singular = 0;
    unsigned ngroup = 0;

    for (int64_t it = blockIdx.x; it < a.item_count; it += gridDim.x) {
        const int32_t *item = a.items + 3 * (a.item_seg + it);
        const int j = item[0], start = item[1], count = item[2];
        const int64_t nb = a.pb.node_ptr[j];
        for (int k = tid; k < 3 * ND; k += 256) s_cf[k] = a.coef[3 * nb + k];
        for (int k = tid; k < 2 * KS; k += 256) s_sc[k] = k < 2 * ND ? aa.scoef[2 * nb + k] : 0.0;
        const double *cf = s_cf;
        const double tau = a.tau[j];
        const double rho_j = a.rho[j];
        unsigned item_groups = 0;
        if (tid < count) {
            const int p = a.plist[start + tid];
            const int64_t t = a.pair_tgt[p];
            s_x[tid][0] = a.pb.txyz[3 * t];
            s_x[tid][1] = a.pb.txyz[3 * t + 1];
            s_x[tid][2] = a.pb.txyz[3 * t + 2];
            // rounding-floor factor of this target (see kNoiseKappa)
            s_nf[tid] = noise_factor(__builtin_sqrt(s_x[tid][0] * s_x[tid][0] + s_x[tid][1] * s_x[tid][1] +
                                                    s_x[tid][2] * s_x[tid][2]) + rho_j);
            s_lam[tid][0] = aa.lam[2 * t];
            s_lam[tid][1] = -aa.lam[2 * t + 1];  // conj(lambda)
            s_pair[tid] = p;
        }
        for (int k = tid; k < 64 * 6; k += 256) (&s_t[0][0])[k] = 0.0;
        // the chart and density coefficients were staged by every wave
        __syncthreads();
        if (tid < 64)
            node_geometry<D, true, true>(cf, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, a.rule[3 * tid],
                                         a.rule[3 * tid + 1], a.rule[3 * tid + 2],
                                         s_geo + tid * GSA, tid & 15);
        __syncthreads();
        // root moments (as in the forward)
        for (int s = wv; s < count; s += 4) {
            const double x[3] = {s_x[s][0], s_x[s][1], s_x[s][2]};
            double acc[W];
#pragma unroll
            for (int v = 0; v < W; ++v) acc[v] = 0.0;
            const double *g = s_geo + lane * GSA;
            double fr, fi, sn;
            kern_node(a.kern, a.helm, x, g + G0, g[pad_slot<S::R>(l16)], fr, fi, singular, sn);
            mac_node<D, true>(acc, g, fr, fi);
            rot_reduce16<PL>(acc);
#pragma unroll
            for (int i = 0; i < PL; ++i) {
                acc[i] += __shfl_xor(acc[i], 16, 64);
                acc[i] += __shfl_xor(acc[i], 32, 64);
            }
            if (grp16 == 0) {
                double *dst = mptr(0, 0, s);
#pragma unroll
                for (int i = 0; i < PL; ++i) dst[PL * l16 + i] = acc[i];
            }
        }
        if (tid == 0) {
            GroupEntry &e = s_stack[0];
            e.tri[0] = 0.0; e.tri[1] = 0.0; e.tri[2] = 1.0; e.tri[3] = 0.0; e.tri[4] = 0.0; e.tri[5] = 1.0;
            e.level = 0;
            e.child = 0;
            e.mask = count == 64 ? ~0ull : ((1ull << count) - 1ull);
            s_fail2[0] = 0ull;
        }
        __syncthreads();
        // per-wavefront moment vectors (unit l16 of each) and scalar sums
        double GM[9 * PL];
#pragma unroll
        for (int v = 0; v < 9 * PL; ++v) GM[v] = 0.0;
        double SC[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // dPhi/dk, Phi_S, Phi_D
        // stack depth and failing-target words as in the forward kernel
        int sp = 1;
        unsigned gpar = 0;
        while (sp > 0) {
            const GroupEntry e = s_stack[sp - 1];
            --sp;
            unsigned long long *const s_fail = &s_fail2[gpar & 1];
            if (tid == 0) s_fail2[(gpar + 1) & 1] = 0ull;
            const bool capped = ++item_groups > kGroupCap;
            const double ax = e.tri[0], ay = e.tri[1], bx = e.tri[2], by = e.tri[3];
            const double cx = e.tri[4], cy = e.tri[5];
            const double abx = 0.5 * (ax + bx), aby = 0.5 * (ay + by);
            const double bcx = 0.5 * (bx + cx), bcy = 0.5 * (by + cy);
            const double cax = 0.5 * (cx + ax), cay = 0.5 * (cy + ay);
            const double area = __builtin_ldexp(1.0, -2 * (e.level + 1));
            {
                const int c = tid >> 6, q = tid & 63;
                double Ax, Ay, Bx, By, Cx, Cy;
                if (c == 0) { Ax = ax; Ay = ay; Bx = abx; By = aby; Cx = cax; Cy = cay; }
                else if (c == 1) { Ax = abx; Ay = aby; Bx = bx; By = by; Cx = bcx; Cy = bcy; }
                else if (c == 2) { Ax = cax; Ay = cay; Bx = bcx; By = bcy; Cx = cx; Cy = cy; }
                else { Ax = bcx; Ay = bcy; Bx = cax; By = cay; Cx = abx; Cy = aby; }
                node_geometry<D, true, true>(cf, Ax, Ay, Bx, By, Cx, Cy, a.rule[3 * q],
                                             a.rule[3 * q + 1], a.rule[3 * q + 2] * area,
                                             s_geo + tid * GSA, tid & 15);
            }
            // a single-target group reads only each thread's own node row
            if (__builtin_popcountll(e.mask) != 1) __syncthreads();
            const double thr = tau * __builtin_ldexp(1.0, -2 * e.level);
            const int L = e.level;
            // ---- the forward's work split and test, in the same arithmetic
            const int kofs = (int)((ngroup++ + blockIdx.x) & 3);
            if (__builtin_popcountll(e.mask) == 1) {
                const int s = __builtin_ctzll(e.mask);
                const double x[3] = {s_x[s][0], s_x[s][1], s_x[s][2]};
                double IT[PL];
                {
                    const double *src = mptr(L, e.child, s);
#pragma unroll
                    for (int i = 0; i < PL; ++i) IT[i] = src[PL * l16 + i];
                }
                double acc[W];
#pragma unroll
                for (int v = 0; v < W; ++v) acc[v] = 0.0;
                double sens;
                {
                    const double *g = s_geo + tid * GSA;
                    double fr, fi;
                    kern_node(a.kern, a.helm, x, g + G0, g[pad_slot<S::R>(l16)], fr, fi, singular, sens);
                    mac_node<D, true>(acc, g, fr, fi);
                }
                sens = wave_total(sens);
                if (lane == 0) s_g2[wv] = sens;
                rot_reduce16<PL>(acc);
                double cm[PL];
#pragma unroll
                for (int i = 0; i < PL; ++i) {
                    double v = acc[i] + __shfl_xor(acc[i], 16, 64);
                    v += __shfl_xor(v, 32, 64);
                    cm[i] = v;
                    if (grp16 == 0) s_cm[wv * W + PL * l16 + i] = v;
                }
                __syncthreads();
                double e2 = 0.0;
#pragma unroll
                for (int i = 0; i < PL; ++i) {
                    const int o = PL * l16 + i;
                    const double v = (s_cm[o] + s_cm[W + o]) + (s_cm[2 * W + o] + s_cm[3 * W + o]);
                    const double df = v - IT[i];
                    if (PL * l16 + i < S::NV) e2 = __builtin_fma(df, df, e2);
                }
                const double err2 = lane0(row_sum16(e2));
                const double noise2 = s_nf[s] * ((s_g2[0] + s_g2[1]) + (s_g2[2] + s_g2[3]));
                bool accept = (err2 <= thr * thr || err2 <= noise2) && L + 1 >= a.min_depth;
                if (!accept && (L + 1 >= a.max_depth || capped)) accept = true;
                if (!accept) {
                    if (grp16 == 0) {
                        double *dst = mptr(L + 1, wv, s);
#pragma unroll
                        for (int i = 0; i < PL; ++i) dst[PL * l16 + i] = cm[i];
                    }
                    if (tid == 0) *s_fail = 1ull << s;
                }
            } else {
                unsigned long long mk = e.mask;
                int k = kofs;
                while (mk) {
                    const int s = __builtin_ctzll(mk);
                    mk &= mk - 1ull;
                    if ((k++ & 3) != wv) continue;
                    const double x[3] = {s_x[s][0], s_x[s][1], s_x[s][2]};
                    double IT[PL];
                    {
                        const double *src = mptr(L, e.child, s);
#pragma unroll
                        for (int i = 0; i < PL; ++i) IT[i] = src[PL * l16 + i];
                    }
                    double acc[W];
#pragma unroll
                    for (int v = 0; v < W; ++v) acc[v] = 0.0;
                    double sens = 0.0;
#pragma unroll 1
                    for (int i = 0; i < 4; ++i) {
                        const double *g = s_geo + (grp16 * 64 + l16 + 16 * i) * GSA;
                        double fr, fi, sn;
                        kern_node(a.kern, a.helm, x, g + G0, g[pad_slot<S::R>(l16)], fr, fi, singular, sn);
                        mac_node<D, true>(acc, g, fr, fi);
                        sens += sn;
                    }
                    rot_reduce16<PL>(acc);
                    double e2 = 0.0;
#pragma unroll
                    for (int i = 0; i < PL; ++i) {
                        double v = acc[i] + __shfl_xor(acc[i], 16, 64);
                        v += __shfl_xor(v, 32, 64);
                        const double df = v - IT[i];
                        if (PL * l16 + i < S::NV) e2 = __builtin_fma(df, df, e2);
                    }
                    const double err2 = lane0(row_sum16(e2));
                    bool accept = (err2 <= thr * thr || err2 <= s_nf[s] * wave_total(sens)) &&
                                  L + 1 >= a.min_depth;
                    if (!accept && (L + 1 >= a.max_depth || capped)) accept = true;
                    if (!accept) {
                        double *dst = mptr(L + 1, grp16, s);
#pragma unroll
                        for (int i = 0; i < PL; ++i) dst[PL * l16 + i] = acc[i];
                        if (lane == 0) atomicOr(s_fail, 1ull << s);
                    }
                }
            }
            __syncthreads();
            // ---- gradient over the children nodes for the accepting targets
            const unsigned long long accm = e.mask & ~*s_fail;
            if (accm != 0ull) {
                const double *g = s_geo + tid * GSA;
                const double X[3] = {g[G0], g[G0 + 1], g[G0 + 2]};
                const double Xu[3] = {g[G0 + 7], g[G0 + 8], g[G0 + 9]};
                const double Xv[3] = {g[G0 + 10], g[G0 + 11], g[G0 + 12]};
                const double n[3] = {Xu[1] * Xv[2] - Xu[2] * Xv[1], Xu[2] * Xv[0] - Xu[0] * Xv[2],
                                     Xu[0] * Xv[1] - Xu[1] * Xv[0]};
                const double wq = a.rule[3 * (tid & 63) + 2] * area;
                // sigma(y) from the rotated basis slots
                double sgr = 0.0, sgi = 0.0;
#pragma unroll
                for (int p = 0; p < 16; ++p)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int m = ((l16 + p) & 15) * R + r;
                        const double kv = g[p * R + r];
                        sgr = __builtin_fma(s_sc[2 * m], kv, sgr);
                        sgi = __builtin_fma(s_sc[2 * m + 1], kv, sgi);
                    }
                double gX[6] = {0, 0, 0, 0, 0, 0}, gn[6] = {0, 0, 0, 0, 0, 0};
                unsigned long long mk = accm;
                int buf = 0;
                while (mk) {
                    const int s = __builtin_ctzll(mk);
                    mk &= mk - 1ull;
                    const double x[3] = {s_x[s][0], s_x[s][1], s_x[s][2]};
                    double rhr, rhi;
                    cmul(s_lam[s][0], s_lam[s][1], sgr, sgi, rhr, rhi);
                    NodeGrad gg;
                    node_grad(a.kern, x, X, n, wq, rhr, rhi, gg);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        gX[2 * c] += gg.gXr[c];
                        gX[2 * c + 1] += gg.gXi[c];
                        gn[2 * c] += gg.gnr[c];
                        gn[2 * c + 1] += gg.gni[c];
                    }
                    SC[0] += gg.gkr; SC[1] += gg.gki;
                    SC[2] += gg.sr; SC[3] += gg.si;
                    SC[4] += gg.dr; SC[5] += gg.di;
                    // target gradient: -sum of gX over the 256 nodes
#pragma unroll
                    for (int v = 0; v < 6; ++v) {
                        const double tv = wave_total(v & 1 ? gg.gXi[v >> 1] : gg.gXr[v >> 1]);
                        if (lane == 0) s_tw[buf][wv][v] = tv;
                    }
                    __syncthreads();
                    if (tid < 6)
                        s_t[s][tid] -= (s_tw[buf][0][tid] + s_tw[buf][1][tid]) +
                                       (s_tw[buf][2][tid] + s_tw[buf][3][tid]);
                    buf ^= 1;
                }
                // nine moment vectors of this wavefront's 64 nodes
                double bv[6], dv[6];
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    const double g0 = gn[ri], g1 = gn[2 + ri], g2 = gn[4 + ri];
                    bv[ri] = Xv[1] * g2 - Xv[2] * g1;
                    bv[2 + ri] = Xv[2] * g0 - Xv[0] * g2;
                    bv[4 + ri] = Xv[0] * g1 - Xv[1] * g0;
                    dv[ri] = g1 * Xu[2] - g2 * Xu[1];
                    dv[2 + ri] = g2 * Xu[0] - g0 * Xu[2];
                    dv[4 + ri] = g0 * Xu[1] - g1 * Xu[0];
                }
#pragma unroll
                for (int v = 0; v < 9; ++v) {
                    const double *f = v < 3 ? gX : (v < 6 ? bv : dv);
                    const int c = v % 3;
                    double acc[W];
#pragma unroll
                    for (int i = 0; i < W; ++i) acc[i] = 0.0;
                    mac_node<D, true>(acc, g, f[2 * c], f[2 * c + 1]);
                    rot_reduce16<PL>(acc);
#pragma unroll
                    for (int i = 0; i < PL; ++i) {
                        double t = acc[i] + __shfl_xor(acc[i], 16, 64);
                        t += __shfl_xor(t, 32, 64);
                        GM[v * PL + i] += t;
                    }
                }
            }
            __syncthreads();
            const unsigned long long fail = *s_fail;
            if (tid == 0 && fail != 0ull) {
                for (int c = 3; c >= 0; --c) {
                    GroupEntry &ne = s_stack[sp + 3 - c];
                    double t0x, t0y, t1x, t1y, t2x, t2y;
                    if (c == 0) { t0x = ax; t0y = ay; t1x = abx; t1y = aby; t2x = cax; t2y = cay; }
                    else if (c == 1) { t0x = abx; t0y = aby; t1x = bx; t1y = by; t2x = bcx; t2y = bcy; }
                    else if (c == 2) { t0x = cax; t0y = cay; t1x = bcx; t1y = bcy; t2x = cx; t2y = cy; }
                    else { t0x = bcx; t0y = bcy; t1x = cax; t1y = cay; t2x = abx; t2y = aby; }
                    ne.tri[0] = t0x; ne.tri[1] = t0y; ne.tri[2] = t1x; ne.tri[3] = t1y;
                    ne.tri[4] = t2x; ne.tri[5] = t2y;
                    ne.level = L + 1;
                    ne.child = c;
                    ne.mask = fail;
                }
            }
            if (fail != 0ull) sp += 4;
            ++gpar;
            __syncthreads();
        }
        // per-wavefront parts to LDS (over the geometry rows, free here), then
        // the four in order
        double (*s_gw)[9 * PL * 16 + 6] = reinterpret_cast<double (*)[9 * PL * 16 + 6]>(s_geo);
        static_assert(4 * (9 * PL * 16 + 6) <= 256 * GSA, "reduction buffer exceeds the geometry rows");
        if (grp16 == 0) {
#pragma unroll
            for (int v = 0; v < 9; ++v)
#pragma unroll
                for (int i = 0; i < PL; ++i) s_gw[wv][v * PL * 16 + PL * l16 + i] = GM[v * PL + i];
        }
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            const double tv = wave_total(SC[v]);
            if (lane == 0) s_gw[wv][9 * PL * 16 + v] = tv;
        }
        __syncthreads();
        {
            const int64_t chunk = aa.cptr[j] + (start - aa.pptr[j]) / 64;
            double *dst = aa.gc_item + chunk * aa.gc_pitch;
            // row: 6 scalars (dPhi/dk, Phi_S, Phi_D), then the moment vectors
            // dst[6 + v * 2 ND + comp], comp < 2 ND
            if (tid < 6) {
                const int o = 9 * PL * 16 + tid;
                dst[tid] = (s_gw[0][o] + s_gw[1][o]) + (s_gw[2][o] + s_gw[3][o]);
            }
            for (int k2 = tid; k2 < 9 * 2 * ND; k2 += 256) {
                const int v = k2 / (2 * ND), comp = k2 - v * 2 * ND;
                const int o = v * PL * 16 + comp;
                dst[6 + k2] = (s_gw[0][o] + s_gw[1][o]) + (s_gw[2][o] + s_gw[3][o]);
            }
            for (int k2 = tid; k2 < count * 6; k2 += 256) {
                const int s = k2 / 6, v = k2 - s * 6;
                aa.t_pair[(int64_t)s_pair[s] * 12 + v] = s_t[s][v];
            }
        }
        __syncthreads();
    }
    singular = wave_or(singular);
    if (lane == 0 && singular) a.flags[kFlagSingular] = 1;
}

// Self pairs: the forward's target-split rule, differentiated with the rule
// (split points, sinh grading) held fixed.  One wavefront per self target.
// The rule nodes go 64 at a time, one per lane: a lane evaluates the chart,
// the density and the kernel derivatives at its node and leaves in LDS the
// eighteen weighted terms f = gX, b = Xv x gn, d = gn x Xu (complex
// 3-vectors) and the basis values K.  The moments M[f]_m = sum_q f(q) K_m(q)
// are accumulated transposed: lane (m mod 16, g) takes basis functions
// m mod 16 + 16 r and the nodes q = g (mod 4), and the four node classes are
// summed at the end.  The chart-coefficient gradient then follows from the
// basis differentiation matrices, as in the patch adjoint:
//     GC[c][a] = M[gX_c]_a + sum_m Du[a][m] M[b_c]_m + Dv[a][m] M[d_c]_m.
// The LDS footprint (K rows only) leaves room for two wavefronts per SIMD.
template <int D>
__global__ __launch_bounds__(64) void k_adjoint_self(AdjArgs aa)
{
    constexpr int ND = nd_of(D);
    constexpr int R = (ND + 15) / 16;
    constexpr int KP = 16 * R + 1;       // LDS doubles per node row of K (odd pitch)
    constexpr int FP = 19;               // LDS doubles per node row of the weighted terms
    __shared__ double s_pan[6][kPanW];
    // chart and density coefficients, read at every node (kept out of registers)
    __shared__ double s_cs[5 * ND];
    __shared__ double s_k[64 * KP];
    __shared__ double s_f[64 * FP];
    const QuadArgs &a = aa.qa;
    const int lane = threadIdx.x & 63;
    const int a16 = lane & 15, grp = lane >> 4;
    const int nr = a.nr, na = a.na;
    for (int64_t idx = blockIdx.x; idx < a.count; idx += gridDim.x) {
        const int p = __builtin_amdgcn_readfirstlane(a.grp[a.seg + idx]);
        if (p < 0) continue;
        const int t = __builtin_amdgcn_readfirstlane(a.pair_tgt[p]);
        const int j = __builtin_amdgcn_readfirstlane(a.pair_patch[p]);
        const int64_t nb = a.pb.node_ptr[j];
        const int64_t node = a.pb.node_of_target[t];
        const int l = (int)(node - nb);
        // chart relative to its constant term, as in the forward self kernel
        for (int k = lane; k < 3 * ND; k += 64) s_cs[k] = a.coef_rel[3 * nb + k];
        for (int k = lane; k < 2 * ND; k += 64) s_cs[3 * ND + k] = aa.scoef[2 * nb + k];
        __syncthreads();
        const double lr = aa.lam[2 * t], li = -aa.lam[2 * t + 1];
        const double tu = a.tab.uv[D][2 * l], tv = a.tab.uv[D][2 * l + 1];
        double x[3], G00, G01, G11;
        {
            double K[ND], Xu[3], Xv[3];
            chart_eval<D>(s_cs, tu, tv, K, x, Xu, Xv);
            G00 = Xu[0] * Xu[0] + Xu[1] * Xu[1] + Xu[2] * Xu[2];
            G01 = Xu[0] * Xv[0] + Xu[1] * Xv[1] + Xu[2] * Xv[2];
            G11 = Xv[0] * Xv[0] + Xv[1] * Xv[1] + Xv[2] * Xv[2];
        }
        // panels exactly as in the forward self kernel
        int npan = 0;
        const double Pv[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const double Ax = Pv[e][0], Ay = Pv[e][1];
            const double Ex = Pv[(e + 1) % 3][0] - Ax, Ey = Pv[(e + 1) % 3][1] - Ay;
            const double EGE = G00 * Ex * Ex + 2.0 * G01 * Ex * Ey + G11 * Ey * Ey;
            const double L = __builtin_sqrt(EGE);
            const double rx = tu - Ax, ry = tv - Ay;
            const double mu = (G00 * rx * Ex + G01 * (rx * Ey + ry * Ex) + G11 * ry * Ey) / EGE;
            const double fx = Ax + mu * Ex - tu, fy = Ay + mu * Ey - tv;
            const double h = __builtin_sqrt(G00 * fx * fx + 2.0 * G01 * fx * fy + G11 * fy * fy);
            const double det = __builtin_fabs((Ax - tu) * Ey - (Ay - tv) * Ex);
            const double x0 = asinh(-mu * L / h), x1 = asinh((1.0 - mu) * L / h);
            const bool split = mu > 0.0 && mu < 1.0;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                if (half == 1 && !split) break;
                if (lane == 0) {
                    double *pp = s_pan[npan];
                    pp[0] = Ax; pp[1] = Ay; pp[2] = Ex; pp[3] = Ey;
                    pp[4] = mu; pp[5] = h / L; pp[6] = det;
                    pp[7] = split ? (half == 0 ? x0 : 0.0) : x0;
                    pp[8] = split ? (half == 0 ? 0.0 : x1) : x1;
                }
                ++npan;
            }
        }
        __syncthreads();
        // acc[r][18]: moments of the eighteen terms for basis a16 + 16 r over
        // this lane's node class
        double acc[R][18];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < 18; ++v) acc[r][v] = 0.0;
        double T12[12];
#pragma unroll
        for (int v = 0; v < 12; ++v) T12[v] = 0.0;
        const int per_panel = na * nr;
        const int total = npan * per_panel;
        const float inv_pp = 1.0f / (float)per_panel, inv_nr = 1.0f / (float)nr;
        for (int base = 0; base < total; base += 64) {
            const int q = base + lane;
            double *kr = s_k + lane * KP;
            double *fr = s_f + lane * FP;
            if (q < total) {
                const int pi = (int)(((float)q + 0.5f) * inv_pp);
                const int rem = q - pi * per_panel;
                const int ia = (int)(((float)rem + 0.5f) * inv_nr), ir = rem - ia * nr;
                const double *pp = s_pan[pi];
                const double Ax = pp[0], Ay = pp[1], Ex = pp[2], Ey = pp[3], mu = pp[4];
                const double hl = pp[5], det = pp[6], xa = pp[7], xb = pp[8];
                const double xi = xa + (xb - xa) * a.gla[2 * ia];
                // sinh and cosh from one exponential (lam needs absolute accuracy)
                const double ex = exp(xi), exi = 1.0 / ex;
                const double lam = mu + hl * (0.5 * (ex - exi));
                const double dlam = hl * (0.5 * (ex + exi)) * (xb - xa) * a.gla[2 * ia + 1];
                const double s = a.glr[2 * ir], ws = a.glr[2 * ir + 1];
                const double dx = Ax + lam * Ex - tu, dy = Ay + lam * Ey - tv;
                const double u = tu + s * dx, v = tv + s * dy;
                // chart, density and basis rows in one recurrence pass
                double X[3] = {0.0, 0.0, 0.0}, Xu[3] = {0.0, 0.0, 0.0}, Xv[3] = {0.0, 0.0, 0.0};
                double sgr = 0.0, sgi = 0.0;
                const double *cs = s_cs;
                asm volatile("" : "+v"(cs));
                koorn_visit<D>(u, v, [&](int m, double k, double ku, double kv) {
                    kr[m] = k;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const double cf = cs[c * ND + m];
                        X[c] = __builtin_fma(cf, k, X[c]);
                        Xu[c] = __builtin_fma(cf, ku, Xu[c]);
                        Xv[c] = __builtin_fma(cf, kv, Xv[c]);
                    }
                    sgr = __builtin_fma(cs[3 * ND + 2 * m], k, sgr);
                    sgi = __builtin_fma(cs[3 * ND + 2 * m + 1], k, sgi);
                });
                const double n[3] = {Xu[1] * Xv[2] - Xu[2] * Xv[1], Xu[2] * Xv[0] - Xu[0] * Xv[2],
                                     Xu[0] * Xv[1] - Xu[1] * Xv[0]};
                double rhr, rhi;
                cmul(lr, li, sgr, sgi, rhr, rhi);
                NodeGrad g;
                node_grad(a.kern, x, X, n, s * det * ws * dlam, rhr, rhi, g);
                // weighted terms: gX, b = Xv x gn, d = gn x Xu; (c, re/im) order
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
                    fr[2 * c] = g.gXr[c];
                    fr[2 * c + 1] = g.gXi[c];
                    fr[6 + 2 * c] = Xv[c1] * g.gnr[c2] - Xv[c2] * g.gnr[c1];
                    fr[6 + 2 * c + 1] = Xv[c1] * g.gni[c2] - Xv[c2] * g.gni[c1];
                    fr[12 + 2 * c] = g.gnr[c1] * Xu[c2] - g.gnr[c2] * Xu[c1];
                    fr[12 + 2 * c + 1] = g.gni[c1] * Xu[c2] - g.gni[c2] * Xu[c1];
                    T12[2 * c] -= g.gXr[c];
                    T12[2 * c + 1] -= g.gXi[c];
                }
                T12[6] += g.gkr;
                T12[7] += g.gki;
                T12[8] += g.sr;
                T12[9] += g.si;
                T12[10] += g.dr;
                T12[11] += g.di;
            } else {
#pragma unroll
                for (int v = 0; v < 18; ++v) fr[v] = 0.0;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            // transposed accumulation over the nodes of this lane's class
            const int nq = total - base < 64 ? total - base : 64;
            for (int i = grp; i < nq; i += 4) {
                const double *f = s_f + i * FP;
                const double *kb = s_k + i * KP;
                double fv[18];
#pragma unroll
                for (int v = 0; v < 18; ++v) fv[v] = f[v];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const double k = kb[a16 + 16 * r];
#pragma unroll
                    for (int v = 0; v < 18; ++v) acc[r][v] = __builtin_fma(fv[v], k, acc[r][v]);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        // sum the four node classes; lanes of class 0 leave M[v][m] in LDS
        double *sm = s_k;   // [18][ND], free after the last chunk
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int v = 0; v < 18; ++v) {
                double w = acc[r][v] + __shfl_xor(acc[r][v], 16, 64);
                w += __shfl_xor(w, 32, 64);
                const int m = a16 + 16 * r;
                if (grp == 0 && m < ND) sm[v * ND + m] = w;
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // GC[(c * ND + a) * 2 + re/im] = M[gX] + Du M[b] + Dv M[d]; v = 2 c + re/im
        {
            double *dst = aa.gc_self + node * aa.self_pitch;
            const double *Du = a.tab.D[D], *Dv = a.tab.D[D] + ND * ND;
            for (int o = lane; o < 6 * ND; o += 64) {
                const int v = o / ND, m0 = o - v * ND;
                double w = sm[v * ND + m0];
                const double *mb = sm + (6 + v) * ND, *md = sm + (12 + v) * ND;
                for (int m = 0; m < ND; ++m)
                    w = __builtin_fma(Du[m0 * ND + m], mb[m], __builtin_fma(Dv[m0 * ND + m], md[m], w));
                dst[2 * ((v >> 1) * ND + m0) + (v & 1)] = w;
            }
        }
#pragma unroll
        for (int v = 0; v < 12; ++v) {
            const double tv2 = wave_sum(T12[v]);
            if (lane == 0) aa.t_pair[(int64_t)p * 12 + v] = tv2;
        }
        // the next pair overwrites s_pan and s_cs
        __syncthreads();
    }
}

// sigma coefficients per patch: s = V sigma_j (complex).
__global__ void k_sigma_coef(Problem pb, DegTab tab, const double *sigma, double *scoef)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= pb.P) return;
    const int d = pb.degree[j];
    const int nd = nd_of(d);
    const double *V = tab.V[d];
    const int64_t nb = pb.node_ptr[j];
    for (int a = 0; a < nd; ++a) {
        double sr = 0.0, si = 0.0;
        for (int l = 0; l < nd; ++l) {
            sr = __builtin_fma(V[a * nd + l], sigma[2 * (nb + l)], sr);
            si = __builtin_fma(V[a * nd + l], sigma[2 * (nb + l) + 1], si);
        }
        scoef[2 * (nb + a)] = sr;
        scoef[2 * (nb + a) + 1] = si;
    }
}

// Node gradients from the chart-coefficient gradients: per patch, sum the
// work-item parts (chunk order) and the self parts (node order), then
// grad_l,c = sum_a V_(a),l G_c,a.
__global__ void k_adj_patch_final(Problem pb, DegTab tab, const int64_t *cptr,
                                  const int64_t *nchunk, const double *gc_item, int item_pitch,
                                  const double *gc_self, int self_pitch,
                                  const unsigned int *is_self_node, double *grad)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= pb.P) return;
    const int d = pb.degree[j];
    const int nd = nd_of(d);
    const double *V = tab.V[d];
    const double *Du = tab.D[d], *Dv = tab.D[d] + nd * nd;
    const int64_t nb = pb.node_ptr[j];
    double G[6 * kNDMax];
    for (int v = 0; v < 6 * nd; ++v) G[v] = 0.0;
    // work items in chunk order: dPhi/dchi_c = M[gX_c] + Du M[b_c] + Dv M[d_c]
    for (int64_t c = 0; c < nchunk[j]; ++c) {
        const double *M = gc_item + (cptr[j] + c) * item_pitch + 6;
        for (int cc = 0; cc < 3; ++cc)
            for (int a = 0; a < nd; ++a) {
                const double *Mx = M + cc * 2 * nd, *Mb = M + (3 + cc) * 2 * nd;
                const double *Md = M + (6 + cc) * 2 * nd;
                double gr = Mx[2 * a], gi = Mx[2 * a + 1];
                for (int m = 0; m < nd; ++m) {
                    gr = __builtin_fma(Du[a * nd + m], Mb[2 * m], gr);
                    gi = __builtin_fma(Du[a * nd + m], Mb[2 * m + 1], gi);
                    gr = __builtin_fma(Dv[a * nd + m], Md[2 * m], gr);
                    gi = __builtin_fma(Dv[a * nd + m], Md[2 * m + 1], gi);
                }
                G[2 * (cc * nd + a)] += gr;
                G[2 * (cc * nd + a) + 1] += gi;
            }
    }
    for (int l = 0; l < nd; ++l) {
        if (!is_self_node[nb + l]) continue;
        const double *src = gc_self + (nb + l) * self_pitch;
        for (int v = 0; v < 6 * nd; ++v) G[v] += src[v];
    }
    for (int l = 0; l < nd; ++l)
        for (int c = 0; c < 3; ++c) {
            double gr = 0.0, gi = 0.0;
            for (int a = 0; a < nd; ++a) {
                const double vv = V[a * nd + l];
                gr = __builtin_fma(vv, G[2 * (c * nd + a)], gr);
                gi = __builtin_fma(vv, G[2 * (c * nd + a) + 1], gi);
            }
            grad[2 * (3 * (nb + l) + c)] = gr;
            grad[2 * (3 * (nb + l) + c) + 1] = gi;
        }
}

// Target gradients: for node targets, add the row's pair parts in row order.
__global__ void k_adj_target_final(Problem pb, const int64_t *pair_ptr, const double *t_pair,
                                   double *grad)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= pb.NT) return;
    const int64_t node = pb.node_of_target[t];
    if (node < 0) return;
    double g[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t p = pair_ptr[t]; p < pair_ptr[t + 1]; ++p)
        for (int v = 0; v < 6; ++v) g[v] += t_pair[p * 12 + v];
    for (int v = 0; v < 6; ++v) grad[6 * node + v] += g[v];
}

// dPhi/dk, dPhi/dalpha = Phi_S, dPhi/dbeta = Phi_D: fixed-order block sum
// over the pairs.
__global__ __launch_bounds__(256) void k_adj_scalars(int64_t np, const double *t_pair,
                                                     int64_t nitems, const double *gc_item,
                                                     int item_pitch, double *grad_k, double *dphi)
{
    __shared__ double s[256][6];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    // self pairs carry theirs per pair, near work items per item
    for (int64_t p = threadIdx.x; p < np; p += 256)
        for (int v = 0; v < 6; ++v) acc[v] += t_pair[p * 12 + 6 + v];
    for (int64_t c = threadIdx.x; c < nitems; c += 256)
        for (int v = 0; v < 6; ++v) acc[v] += gc_item[c * item_pitch + v];
    for (int v = 0; v < 6; ++v) s[threadIdx.x][v] = acc[v];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int v = 0; v < 6; ++v) s[threadIdx.x][v] += s[threadIdx.x + w][v];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        grad_k[0] = s[0][0];
        grad_k[1] = s[0][1];
        if (dphi)
            for (int v = 0; v < 4; ++v) dphi[v] = s[0][2 + v];
    }
}

// Marks the nodes that are targets (their self parts exist); two targets on
// one node are rejected (the target-gradient pass writes each node once).
__global__ void k_mark_self_nodes(Problem pb, unsigned int *mark, int *flags)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= pb.NT) return;
    const int64_t node = pb.node_of_target[t];
    if (node < 0 || node >= pb.N) return;
    if (atomicAdd(&mark[node], 1u) > 0u) flags[kFlagInvalid] = 1;
}

}  // namespace nfq
