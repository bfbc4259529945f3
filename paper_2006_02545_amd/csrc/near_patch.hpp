// near_patch.hpp -- patch-centric adaptive near quadrature (Section 4.3 of
// the paper, with its reuse of subtriangle geometry across targets).
//
// One workgroup (4 wavefronts) owns one work item: a patch and up to 64 of
// the targets in its near field.  It walks the union of the targets'
// subdivision trees depth first.  A tree node ("group") is a subtriangle T
// of T0 together with the set of targets (a 64-bit mask) whose test on T is
// pending.  For a group the workgroup
//   1. evaluates the chart at the 4 x 64 rule nodes of T's four children
//      once (256 threads, one node each) and keeps position, weighted normal,
//      weighted Jacobian and Koornwinder values in LDS;
//   2. lets every wavefront take targets of the mask in turn: 16 lanes per
//      child, 4 nodes per lane, kernel values times basis values accumulated
//      in registers, then a 16-lane reduce-scatter (shuffles) that leaves
//      every lane with a few components of the child's moments;
//   3. applies the test ||I_T - sum I_C|| <= tau |T|/|T0|: a target that
//      passes adds sum I_C to its output block; a failing target stores its
//      four child moment vectors for the next level and joins the children's
//      mask.
// Output blocks are accumulated in depth-first order with one wavefront per
// target and group, so the result does not depend on scheduling.
#pragma once

#include "kernels.hpp"

namespace nfq {

constexpr int kGroupStack = 3 * kMaxDepth + 8;

// Moments are reduced over the 16 lanes of a row by rotations (DPP row_ror):
// the ND basis functions are padded to KS = 16 R slots, grouped into 16 units
// of R; the lane with row index l stores unit (l + p) mod 16 in its slot
// group p, so that the reduce-scatter needs no per-lane selects and leaves
// unit l (R functions, times 1 or 2 for complex) on lane l.
template <int D, bool CPLX>
struct PatchShape {
    static constexpr int ND = nd_of(D);
    static constexpr int C = CPLX ? 2 : 1;           // doubles per moment
    static constexpr int NV = C * ND;                // doubles per moment vector
    static constexpr int R = (ND + 15) / 16;         // basis functions per unit
    static constexpr int KS = 16 * R;                // basis slots per node
    static constexpr int PL = R * C;                 // doubles per lane after the reduce-scatter
    static constexpr int W = 16 * PL;                // doubles per lane before it
    static constexpr int GS = (KS + 7) | 1;          // LDS doubles per node (odd pitch)
    static constexpr int G0 = KS;                    // y, n w, J w follow the basis slots
    // The last basis slot (index KS - 1 >= ND) is padding; it carries |K|^2
    // of the node instead of zero.  The moment component it feeds (>= NV) is
    // kept out of the test and of the output.
    // per-target totals kept in LDS when they fit beside the geometry
    static constexpr bool TOT_LDS = (64 * NV + 256 * GS) * 8 <= 140 * 1024;
    static constexpr int TOTN = TOT_LDS ? 64 * NV : 1;
};

// Rotated position of the padding slot for reader row lane l16.
template <int R>
__device__ __forceinline__ int pad_slot(int l16)
{
    return ((15 - l16) & 15) * R + R - 1;
}

// Doubles per lane of the moment vectors for degree d (host sizing).
inline constexpr int patch_w(int d, bool cplx)
{
    return 16 * ((nd_of(d) + 15) / 16) * (cplx ? 2 : 1);
}

struct PatchArgs {
    Problem pb;
    DegTab tab;
    Kern kern;
    int helm;
    int max_depth;
    int min_depth;            // checks above this depth always refine
    const double *rule;       // [64][3]
    const int32_t *items;     // [n][3]: patch, start in plist, count (<= 64)
    int64_t item_seg, item_count;
    const int32_t *plist;     // near pairs in patch-major order
    const int32_t *pair_tgt;
    const int64_t *pair_off;
    const double *coef;
    const double *tau;
    const double *rho;        // max_l |x_l| per patch (coordinate scale)
    double *val;
    double *mom;              // per workgroup slot: [max_depth + 1][4][64][W]
    int64_t mom_slot;         // doubles per slot
    int *flags;
    unsigned long long *stats;
};

// Value of lane (l - N) mod 16 of the same row (DPP row rotation).
template <int N>
__device__ __forceinline__ double row_ror(double x)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, 0x120 + N, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), 0x120 + N, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Reduce-scatter over the 16 lanes of each row for the rotated slot layout:
// on entry acc[W] holds this lane's partial sums with slot group p carrying
// unit (l + p) mod 16; on exit acc[0..PL) holds unit l summed over the row.
template <int PL>
__device__ __forceinline__ void rot_reduce16(double *acc)
{
#pragma unroll
    for (int i = 0; i < 8 * PL; ++i) acc[i] += row_ror<8>(acc[i + 8 * PL]);
#pragma unroll
    for (int i = 0; i < 4 * PL; ++i) acc[i] += row_ror<4>(acc[i + 4 * PL]);
#pragma unroll
    for (int i = 0; i < 2 * PL; ++i) acc[i] += row_ror<2>(acc[i + 2 * PL]);
#pragma unroll
    for (int i = 0; i < PL; ++i) acc[i] += row_ror<1>(acc[i + PL]);
}

// Sum over the 16 lanes of each row, into every lane of the row.
__device__ __forceinline__ double row_sum16(double v)
{
    v += row_ror<8>(v);
    v += row_ror<4>(v);
    v += row_ror<2>(v);
    v += row_ror<1>(v);
    return v;
}

// Wave-uniform copy of lane 0's value.
__device__ __forceinline__ double lane0(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Geometry of one rule node of triangle (A, B, C) into LDS row g: basis
// values in the rotated slot order of reader row lane l16 (padding slots 0),
// then y, n w, J w.
template <int D, bool CPLX, bool DERIV = false>
__device__ __forceinline__ void node_geometry(const double *cf, double Ax, double Ay, double Bx,
                                              double By, double Cx, double Cy, double ru, double rv,
                                              double wgt, double *g, int l16)
{
    using S = PatchShape<D, CPLX>;
    constexpr int ND = S::ND, R = S::R, G0 = S::G0;
    asm volatile("" : "+v"(ru));
    const double u = Ax + ru * (Bx - Ax) + rv * (Cx - Ax);
    const double v = Ay + ru * (By - Ay) + rv * (Cy - Ay);
    double K[ND], X[3], Xu[3], Xv[3];
    chart_eval<D>(cf, u, v, K, X, Xu, Xv);
    const double n0 = Xu[1] * Xv[2] - Xu[2] * Xv[1];
    const double n1 = Xu[2] * Xv[0] - Xu[0] * Xv[2];
    const double n2 = Xu[0] * Xv[1] - Xu[1] * Xv[0];
    g[G0 + 0] = X[0]; g[G0 + 1] = X[1]; g[G0 + 2] = X[2];
    g[G0 + 3] = n0 * wgt; g[G0 + 4] = n1 * wgt; g[G0 + 5] = n2 * wgt;
    g[G0 + 6] = __builtin_sqrt(n0 * n0 + n1 * n1 + n2 * n2) * wgt;
    double kk2 = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m) kk2 = __builtin_fma(K[m], K[m], kk2);
    if (DERIV) {
        // chart derivatives for the adjoint
        g[G0 + 7] = Xu[0]; g[G0 + 8] = Xu[1]; g[G0 + 9] = Xu[2];
        g[G0 + 10] = Xv[0]; g[G0 + 11] = Xv[1]; g[G0 + 12] = Xv[2];
    }
    int rot = (16 - l16) & 15;
    // keep the slot addresses local to this call (hoisting them out of the
    // caller's loops would pin 16 R registers for the whole kernel)
    asm volatile("" : "+v"(rot));
#pragma unroll
    for (int m = 0; m < 16 * R; ++m) {
        const int unit = m / R, r = m - unit * R;
        g[((unit + rot) & 15) * R + r] = m < ND ? K[m] : (m == 16 * R - 1 ? kk2 : 0.0);
    }
}

// acc += (fr, fi) times the basis slots of node row g.
template <int D, bool CPLX>
__device__ __forceinline__ void mac_node(double *acc, const double *g, double fr, double fi)
{
    using S = PatchShape<D, CPLX>;
#pragma unroll
    for (int m = 0; m < S::KS; ++m) {
        const double kv = g[m];
        if (CPLX) {
            acc[2 * m] = __builtin_fma(fr, kv, acc[2 * m]);
            acc[2 * m + 1] = __builtin_fma(fi, kv, acc[2 * m + 1]);
        } else {
            acc[m] = __builtin_fma(fr, kv, acc[m]);
        }
    }
}

// Weighted kernel value at a node whose geometry g carries n w and J w.
__device__ __forceinline__ void kern_node(const Kern &k, bool helm, const double x[3],
                                          const double *g, double kk2, double &fr, double &fi,
                                          int &singular, double &sens)
{
    // g points at the node's y, n w, J w; sens: rounding sensitivity
    // (|f|^2 / r^2 + b^2) |K|^2 of the weighted value (see kNoiseKappa)
    const double dx = x[0] - g[0], dy = x[1] - g[1], dz = x[2] - g[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) singular = 1;
    const double rinv = rsqrt_nr(r2);
    const double g0 = kInv4Pi * rinv;
    const double gJ = g0 * g[6];
    const double rinv2 = rinv * rinv;
    const double d0 = g0 * (g[3] * dx + g[4] * dy + g[5] * dz) * rinv2;
    const double bs = k.bm * gJ * rinv2;
    if (!helm) {
        fr = k.ar * gJ + k.br * d0;
        fi = k.ai * gJ + k.bi * d0;
        sens = ((fr * fr + fi * fi) * rinv2 + bs * bs) * kk2;
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
    const double pr = 1.0 + k.ki * r, pi = -k.kr * r;
    const double gr = gJ * c, gi = gJ * s;
    const double qr = d0 * (pr * c - pi * s), qi = d0 * (pr * s + pi * c);
    fr = k.ar * gr - k.ai * gi + k.br * qr - k.bi * qi;
    fi = k.ar * gi + k.ai * gr + k.br * qi + k.bi * qr;
    sens = ((fr * fr + fi * fi) * rinv2 + bs * bs) * kk2;
}

// Sum over the wavefront, into every lane (row sums by rotation, then the
// four rows).
__device__ __forceinline__ double wave_total(double v)
{
    v = row_sum16(v);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// Largest number of subdivision groups one work item may take; beyond it the
// remaining tests accept (and count as non-converged).  It bounds the walk
// far above any converging tree.
constexpr unsigned kGroupCap = 1u << 18;

struct GroupEntry {
    double tri[6];
    int level;
    int child;
    unsigned long long mask;
};

template <int D, bool CPLX>
__global__ __launch_bounds__(256, (D <= 4 ? 2 : 1)) void k_near_patch(PatchArgs a)
{
    using S = PatchShape<D, CPLX>;
    constexpr int NV = S::NV, W = S::W, PL = S::PL, GS = S::GS, G0 = S::G0;
    constexpr int C = S::C;
    __shared__ double s_geo[256 * GS];
    __shared__ double s_tot[S::TOTN];
    __shared__ GroupEntry s_stack[kGroupStack];
    __shared__ double s_x[64][3];
    __shared__ int64_t s_off[64];
    __shared__ double s_cf[3 * S::ND];
    __shared__ double s_cm[4 * W];
    __shared__ double s_g2[4];
    __shared__ double s_nf[64];
    // failing-target masks of the current and the next group (alternating)
    __shared__ unsigned long long s_fail2[2];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int grp16 = lane >> 4, l16 = lane & 15;
    double *mom = a.mom + (int64_t)blockIdx.x * a.mom_slot;
    // moments of target slot s, child c at level L: mom[((L * 4 + c) * 64 + s) * W + comp]
    auto mptr = [&](int L, int c, int s) { return mom + ((int64_t)(L * 4 + c) * 64 + s) * W; };
    unsigned long long st_visits = 0, st_checks = 0, st_nonconv = 0, st_maxlev = 0, st_pairs = 0;
    int singular = 0;
    unsigned ngroup = 0;

    for (int64_t it = blockIdx.x; it < a.item_count; it += gridDim.x) {
        const int32_t *item = a.items + 3 * (a.item_seg + it);
        const int j = item[0], start = item[1], count = item[2];
        // chart coefficients in LDS, read at every use (kept out of registers)
        for (int k = tid; k < 3 * S::ND; k += 256) s_cf[k] = a.coef[3 * a.pb.node_ptr[j] + k];
        const double *cf = s_cf;
        const double tau = a.tau[j];
        const double rho_j = a.rho[j];
        // rounding-floor factor of target s (see kNoiseKappa)
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
            const int64_t off = a.pair_off[p];
            s_off[tid] = off;
            if (!S::TOT_LDS)
                for (int v = 0; v < NV; ++v) a.val[C * off + v] = 0.0;
        }
        if (S::TOT_LDS)
            for (int k = tid; k < 64 * NV; k += 256) s_tot[k] = 0.0;
        // the chart coefficients were staged by every wave
        __syncthreads();
        if (tid < 64) {
            // root geometry: node tid of the rule on T0, read by lane tid
            node_geometry<D, CPLX>(cf, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, a.rule[3 * tid],
                                   a.rule[3 * tid + 1], a.rule[3 * tid + 2], s_geo + tid * GS,
                                   tid & 15);
        }
        __syncthreads();
        // root moments of every target: one node per lane
        for (int s = wv; s < count; s += 4) {
            const double x[3] = {s_x[s][0], s_x[s][1], s_x[s][2]};
            double acc[W];
#pragma unroll
            for (int v = 0; v < W; ++v) acc[v] = 0.0;
            const double *g = s_geo + lane * GS;
            double fr, fi, sn;
            kern_node(a.kern, a.helm, x, g + G0, g[pad_slot<S::R>(l16)], fr, fi, singular, sn);
            mac_node<D, CPLX>(acc, g, fr, fi);
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
            ++st_pairs;
            ++st_visits;
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
        // The stack depth is uniform and kept by every thread; tid 0 writes
        // the pushed entries.  Group g collects its failing targets in
        // s_fail2[g & 1] and clears the other word for group g + 1 (whose
        // last readers finished before the previous group's final barrier).
        int sp = 1;
        unsigned gpar = 0;
        while (sp > 0) {
            const GroupEntry e = s_stack[sp - 1];
            --sp;
            unsigned long long *const s_fail = &s_fail2[gpar & 1];
            if (tid == 0) s_fail2[(gpar + 1) & 1] = 0ull;
            const bool capped = ++item_groups > kGroupCap;
            // children geometry: thread tid -> child tid / 64, node tid % 64,
            // read by row lane tid % 16
            const double ax = e.tri[0], ay = e.tri[1], bx = e.tri[2], by = e.tri[3];
            const double cx = e.tri[4], cy = e.tri[5];
            const double abx = 0.5 * (ax + bx), aby = 0.5 * (ay + by);
            const double bcx = 0.5 * (bx + cx), bcy = 0.5 * (by + cy);
            const double cax = 0.5 * (cx + ax), cay = 0.5 * (cy + ay);
            {
                const int c = tid >> 6, q = tid & 63;
                double Ax, Ay, Bx, By, Cx, Cy;
                if (c == 0) { Ax = ax; Ay = ay; Bx = abx; By = aby; Cx = cax; Cy = cay; }
                else if (c == 1) { Ax = abx; Ay = aby; Bx = bx; By = by; Cx = bcx; Cy = bcy; }
                else if (c == 2) { Ax = cax; Ay = cay; Bx = bcx; By = bcy; Cx = cx; Cy = cy; }
                else { Ax = bcx; Ay = bcy; Bx = cax; By = cay; Cx = abx; Cy = aby; }
                const double area = __builtin_ldexp(1.0, -2 * (e.level + 1));
                node_geometry<D, CPLX>(cf, Ax, Ay, Bx, By, Cx, Cy, a.rule[3 * q], a.rule[3 * q + 1],
                                       a.rule[3 * q + 2] * area, s_geo + tid * GS, tid & 15);
            }
            // a single-target group reads only each thread's own node row
            // (wavefront c takes child c, lane q node q): no exchange needed
            if (__builtin_popcountll(e.mask) != 1) __syncthreads();
            const double thr = tau * __builtin_ldexp(1.0, -2 * e.level);
            const int L = e.level;
            // the wavefront that takes the first target of this group (varies
            // from group to group to spread the work over the SIMDs)
            const int kofs = (int)((ngroup++ + blockIdx.x) & 3);
            if (__builtin_popcountll(e.mask) == 1) {
                // one target: the four wavefronts take one child each, one
                // node per lane; children moments meet in LDS
                const int s = __builtin_ctzll(e.mask);
                const bool mine = wv == kofs;
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
                    const double *g = s_geo + tid * GS;
                    double fr, fi;
                    kern_node(a.kern, a.helm, x, g + G0, g[pad_slot<S::R>(l16)], fr, fi, singular, sens);
                    mac_node<D, CPLX>(acc, g, fr, fi);
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
                double Ssum[PL];
                double e2 = 0.0;
#pragma unroll
                for (int i = 0; i < PL; ++i) {
                    const int o = PL * l16 + i;
                    const double v = (s_cm[o] + s_cm[W + o]) + (s_cm[2 * W + o] + s_cm[3 * W + o]);
                    Ssum[i] = v;
                    const double df = v - IT[i];
                    if (PL * l16 + i < S::NV) e2 = __builtin_fma(df, df, e2);
                }
                const double err2 = lane0(row_sum16(e2));
                const double noise2 = s_nf[s] * ((s_g2[0] + s_g2[1]) + (s_g2[2] + s_g2[3]));
                if (mine) {
                    ++st_checks;
                    st_visits += 4;
                }
                const bool ok = err2 <= thr * thr || err2 <= noise2;
                bool accept = ok && L + 1 >= a.min_depth;
                if (!accept && (L + 1 >= a.max_depth || capped)) {
                    accept = true;
                    if (!ok && mine) ++st_nonconv;
                }
                if (accept) {
                    if (mine && grp16 == 0) {
                        double *dst = S::TOT_LDS ? s_tot + s * NV : a.val + C * s_off[s];
#pragma unroll
                        for (int i = 0; i < PL; ++i) {
                            const int comp = PL * l16 + i;
                            if (comp < NV) dst[comp] += Ssum[i];
                        }
                    }
                    if (mine && (unsigned long long)(L + 1) > st_maxlev) st_maxlev = L + 1;
                } else {
                        if (grp16 == 0) {
                            double *dst = mptr(L + 1, wv, s);
#pragma unroll
                            for (int i = 0; i < PL; ++i) dst[PL * l16 + i] = cm[i];
                        }
                        if (tid == 0) *s_fail = 1ull << s;
                    }
                } else {
                // targets of the mask, the k-th set bit to wavefront (k + kofs) % 4
                unsigned long long mk = e.mask;
                int k = kofs;
                while (mk) {
                    const int s = __builtin_ctzll(mk);
                    mk &= mk - 1ull;
                    if ((k++ & 3) != wv) continue;
                    const double x[3] = {s_x[s][0], s_x[s][1], s_x[s][2]};
                    // parent moments: loads issued before the node work
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
                        const double *g = s_geo + (grp16 * 64 + l16 + 16 * i) * GS;
                        double fr, fi, sn;
                        kern_node(a.kern, a.helm, x, g + G0, g[pad_slot<S::R>(l16)], fr, fi, singular, sn);
                        mac_node<D, CPLX>(acc, g, fr, fi);
                        sens += sn;
                    }
                    rot_reduce16<PL>(acc);
                    // acc[0..PL): unit l16 of child grp16's moments; the sum over
                    // the four children by two more exchanges
                    double Ssum[PL];
                    double e2 = 0.0;
#pragma unroll
                    for (int i = 0; i < PL; ++i) {
                        double v = acc[i] + __shfl_xor(acc[i], 16, 64);
                        v += __shfl_xor(v, 32, 64);
                        Ssum[i] = v;
                        const double df = v - IT[i];
                        if (PL * l16 + i < S::NV) e2 = __builtin_fma(df, df, e2);
                    }
                    // every row holds the same children sum: row 0's total decides
                    const double err2 = lane0(row_sum16(e2));
                    ++st_checks;
                    st_visits += 4;
                    // the rounding floor is summed only when the threshold fails
                    const bool ok = err2 <= thr * thr || err2 <= s_nf[s] * wave_total(sens);
                    bool accept = ok && L + 1 >= a.min_depth;
                    if (!accept && (L + 1 >= a.max_depth || capped)) {
                        accept = true;
                        if (!ok) ++st_nonconv;
                    }
                    if (accept) {
                        if (grp16 == 0) {
                            double *dst = S::TOT_LDS ? s_tot + s * NV : a.val + C * s_off[s];
#pragma unroll
                            for (int i = 0; i < PL; ++i) {
                                const int comp = PL * l16 + i;
                                if (comp < NV) dst[comp] += Ssum[i];
                            }
                        }
                        if ((unsigned long long)(L + 1) > st_maxlev) st_maxlev = L + 1;
                    } else {
                        double *dst = mptr(L + 1, grp16, s);
#pragma unroll
                        for (int i = 0; i < PL; ++i) dst[PL * l16 + i] = acc[i];
                        if (lane == 0) atomicOr(s_fail, 1ull << s);
                    }
                }
            }
            __syncthreads();
            const unsigned long long fail = *s_fail;
            if (tid == 0 && fail != 0ull) {
                // push children 3..0 so that child 0 is processed next
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
        if (S::TOT_LDS)
            for (int k = tid; k < count * NV; k += 256) {
                const int s = k / NV, v = k - s * NV;
                a.val[C * s_off[s] + v] = s_tot[k];
            }
        __syncthreads();
    }
    singular = wave_or(singular);
    if (lane == 0) {
        if (singular) a.flags[kFlagSingular] = 1;
        atomicAdd(&a.stats[kStatNear], st_pairs);
        atomicAdd(&a.stats[kStatVisits], st_visits);
        atomicAdd(&a.stats[kStatChecks], st_checks);
        atomicAdd(&a.stats[kStatNonconv], st_nonconv);
        atomicMax(&a.stats[kStatMaxLevel], st_maxlev);
    }
}

// ------------------------------------------------------ work items

// Near pairs per patch.
__global__ void k_patch_count(int64_t np, const int32_t *pair_patch, const int8_t *pair_self,
                              int64_t *pcount)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np || pair_self[p]) return;
    atomicAdd((unsigned long long *)&pcount[pair_patch[p]], 1ull);
}

__global__ void k_patch_chunks(int64_t P, const int64_t *pcount, int64_t *nchunk)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P) return;
    nchunk[j] = (pcount[j] + 63) / 64;
}

// Scatter near pairs into patch-major order.
__global__ void k_patch_scatter(int64_t np, const int32_t *pair_patch, const int8_t *pair_self,
                                const int64_t *pptr, unsigned long long *pcursor, int32_t *plist)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np || pair_self[p]) return;
    const int j = pair_patch[p];
    const unsigned long long k = atomicAdd(&pcursor[j], 1ull);
    plist[pptr[j] + (int64_t)k] = (int32_t)p;
}

// Each patch's near pairs in ascending pair order (that is, by target): the
// scatter above places them in arrival order, and the composition of the
// 64-target work items (hence which tests run split over four wavefronts)
// must not depend on it.  One workgroup per patch; rank sort, from LDS when
// the list fits.
constexpr int kSortLds = 4096;

__global__ __launch_bounds__(256) void k_patch_sort(int64_t P, const int64_t *pptr,
                                                    const int64_t *pcount, const int32_t *raw,
                                                    int32_t *plist)
{
    __shared__ int32_t s_v[kSortLds];
    for (int64_t j = blockIdx.x; j < P; j += gridDim.x) {
        const int64_t n = pcount[j], b = pptr[j];
        const bool lds = n <= kSortLds;
        if (lds)
            for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s_v[i] = raw[b + i];
        __syncthreads();
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            const int32_t v = lds ? s_v[i] : raw[b + i];
            int64_t rank = 0;
            for (int64_t k = 0; k < n; ++k) rank += (lds ? s_v[k] : raw[b + k]) < v;
            plist[b + rank] = v;
        }
        __syncthreads();
    }
}

// Work items (patch, start, count <= 64) into per-degree segments.  Block-
// aggregated: one global atomic per (block, degree).
__global__ __launch_bounds__(256) void k_items(int64_t P, const int32_t *degree,
                                               const int64_t *pcount, const int64_t *pptr,
                                               const int64_t *item_seg_start,
                                               unsigned long long *item_cursor, int32_t *items)
{
    __shared__ unsigned int s_cnt[9];
    __shared__ unsigned long long s_base[9];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (threadIdx.x < 9) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    int d = 0, nch = 0;
    unsigned int local = 0;
    if (j < P) {
        d = degree[j];
        nch = (int)((pcount[j] + 63) / 64);
        if (nch > 0) local = atomicAdd(&s_cnt[d], (unsigned)nch);
    }
    __syncthreads();
    if (threadIdx.x < 9 && s_cnt[threadIdx.x] > 0)
        s_base[threadIdx.x] = atomicAdd(&item_cursor[threadIdx.x], (unsigned long long)s_cnt[threadIdx.x]);
    __syncthreads();
    if (j < P && nch > 0) {
        const int64_t base = item_seg_start[d] + (int64_t)s_base[d] + local;
        for (int c = 0; c < nch; ++c) {
            int32_t *it = items + 3 * (base + c);
            const int64_t st = pptr[j] + 64 * c;
            const int64_t rem = pcount[j] - 64 * c;
            it[0] = (int32_t)j;
            it[1] = (int32_t)st;
            it[2] = (int32_t)(rem < 64 ? rem : 64);
        }
    }
}

}  // namespace nfq
