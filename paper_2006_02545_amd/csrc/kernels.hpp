// kernels.hpp -- HIP kernels of the near-field correction generator.
//
//  * pair / work-queue builder: CSR-by-target row lengths and validation,
//    row and pair pointers (scan), the pair list with output offsets and
//    column indices, grouping of pairs by (degree, near/self);
//  * patch preparation: chart coefficients x_nm = V x_l, d_j, tolerance;
//  * adaptive near quadrature (Section 4.3): one wavefront per pair,
//    depth-first 1->4 midpoint subdivision of T0, 64-point rule per
//    subtriangle, 16 lanes per child triangle;
//  * self quadrature: target-split, Duffy-collapsed tensor Gauss-Legendre
//    with a sinh-graded angular variable in the chart's metric;
//  * moments -> node weights a_l = sum_nm V_(nm),l I_nm (Section 4.3);
//  * sparse apply y = A sigma.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace nfq {

constexpr int kNG = 8;             // subtriangle rule: 8 x 8 conical product
constexpr int kNQ = kNG * kNG;     // 64 nodes = one wavefront
constexpr int kStack = 100;        // DFS stack entries per wavefront (>= 3 max_depth + 4)
constexpr int kMaxDepth = 32;
constexpr int kNDMax = 45;

enum Flag : int {
    kFlagSingular = 0,
    kFlagDegenerate = 1,
    kFlagInvalid = 2,
    kFlagNotRegistered = 3,
    kFlagStackOverflow = 4,
    kNumFlags = 8,
};

enum Stat : int {
    kStatNear = 0, kStatSelf, kStatVisits, kStatChecks, kStatNonconv, kStatMaxLevel, kNumStats = 8,
};

struct DegTab {
    const double *V[9];   // [nd][nd] per degree, V[a * nd + l]
    const double *uv[9];  // [nd][2]
    const double *w[9];   // [nd]
    const double *D[9];   // [2][nd][nd] differentiation matrices in the basis
    double normV[9];
    int present[9];
};

struct Problem {
    int64_t P, N, NT;
    const int32_t *degree;
    const int64_t *node_ptr;
    const double *xyz;
    const double *txyz;
    const int64_t *node_of_target;
    const int64_t *near_rp;
    const int32_t *near_patch;
};

__device__ __forceinline__ int64_t patch_of_node(const int64_t *node_ptr, int64_t P, int64_t node)
{
    int64_t lo = 0, hi = P - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (node_ptr[mid] <= node) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Fills n 32-bit words with v.  The generate sequence clears its counters and
// flags with this kernel rather than with memset nodes, so that it can be
// captured in a graph and replayed.
__global__ __launch_bounds__(256) void k_fill32(int64_t n, uint32_t v, uint32_t *p)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------- builder

// Row lengths of the output CSR and number of (target, patch) blocks per
// row; validates the near list.  counts (optional): blocks per
// (kind * 9 + degree), kind 0 = near, 1 = self.
__global__ void k_rowlen(Problem pb, int present_mask, int64_t *rowlen, int64_t *npair,
                         unsigned long long *counts, int *flags)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= pb.NT) return;
    const int64_t e0 = pb.near_rp[t], e1 = pb.near_rp[t + 1];
    int64_t own = -1;
    const int64_t node = pb.node_of_target[t];
    if (node >= pb.N || node < -1) {
        flags[kFlagInvalid] = 1;
    } else if (node >= 0) {
        own = patch_of_node(pb.node_ptr, pb.P, node);
    }
    int64_t len = 0, cnt = 0;
    if (e1 < e0) {
        flags[kFlagInvalid] = 1;
    } else {
        int64_t prev = -1;
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t j = pb.near_patch[e];
            if (j < 0 || j >= pb.P || j <= prev || j == own) { flags[kFlagInvalid] = 1; break; }
            prev = j;
            const int d = pb.degree[j];
            if (d < 1 || d > 8 || !((present_mask >> d) & 1)) { flags[kFlagNotRegistered] = 1; break; }
            len += nd_of(d);
            ++cnt;
            if (counts) atomicAdd(&counts[d], 1ull);
        }
    }
    if (own >= 0) {
        const int d = pb.degree[own];
        if (d < 1 || d > 8 || !((present_mask >> d) & 1)) {
            flags[kFlagNotRegistered] = 1;
        } else {
            len += nd_of(d);
            ++cnt;
            if (counts) atomicAdd(&counts[9 + d], 1ull);
        }
    }
    rowlen[t] = len;
    npair[t] = cnt;
}

// Exclusive scan of two int64 arrays at once, 1024 items per block;
// writes block totals for the next level.
constexpr int kScanBlock = 256, kScanItems = 4, kScanTile = kScanBlock * kScanItems;

__global__ __launch_bounds__(kScanBlock) void k_scan_tile(int64_t n, const int64_t *a_in,
                                                           const int64_t *b_in, int64_t *a_out,
                                                           int64_t *b_out, int64_t *a_tot,
                                                           int64_t *b_tot)
{
    __shared__ int64_t sa[kScanBlock], sb[kScanBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int64_t va[kScanItems], vb[kScanItems], ra = 0, rb = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t k = base + i;
        va[i] = k < n ? a_in[k] : 0;
        vb[i] = k < n ? b_in[k] : 0;
        ra += va[i];
        rb += vb[i];
    }
    sa[threadIdx.x] = ra;
    sb[threadIdx.x] = rb;
    __syncthreads();
    // Hillis-Steele inclusive scan of thread totals
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int64_t xa = 0, xb = 0;
        if ((int)threadIdx.x >= off) { xa = sa[threadIdx.x - off]; xb = sb[threadIdx.x - off]; }
        __syncthreads();
        sa[threadIdx.x] += xa;
        sb[threadIdx.x] += xb;
        __syncthreads();
    }
    int64_t ea = sa[threadIdx.x] - ra, eb = sb[threadIdx.x] - rb;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t k = base + i;
        if (k < n) { a_out[k] = ea; b_out[k] = eb; }
        ea += va[i];
        eb += vb[i];
    }
    if (threadIdx.x == kScanBlock - 1) {
        a_tot[blockIdx.x] = sa[threadIdx.x];
        b_tot[blockIdx.x] = sb[threadIdx.x];
    }
}

__global__ void k_scan_add(int64_t n, int64_t *a, int64_t *b, const int64_t *a_off,
                           const int64_t *b_off)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t blk = k / kScanTile;
    a[k] += a_off[blk];
    b[k] += b_off[blk];
}

// After the scan: the last entry (n) of the exclusive scans is the total.
__global__ void k_scan_total(int64_t n, const int64_t *a_in, const int64_t *b_in, int64_t *a,
                             int64_t *b)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a[n] = (n > 0 ? a[n - 1] + a_in[n - 1] : 0);
        b[n] = (n > 0 ? b[n - 1] + b_in[n - 1] : 0);
    }
}

// Pair list in row order: target, patch, self flag, output offset; and the
// column indices of every block.
__global__ void k_pairs(Problem pb, const int64_t *row_ptr, const int64_t *pair_ptr,
                        int32_t *pair_tgt, int32_t *pair_patch, int8_t *pair_self,
                        int64_t *pair_off, int32_t *col)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= pb.NT) return;
    const int64_t node = pb.node_of_target[t];
    const int64_t own = node >= 0 ? patch_of_node(pb.node_ptr, pb.P, node) : -1;
    int64_t e = pb.near_rp[t];
    const int64_t e1 = pb.near_rp[t + 1];
    int64_t pos = row_ptr[t], p = pair_ptr[t];
    bool own_done = own < 0;
    while (e < e1 || !own_done) {
        int64_t j;
        bool self = false;
        if (!own_done && (e >= e1 || own < pb.near_patch[e])) { j = own; own_done = true; self = true; }
        else { j = pb.near_patch[e++]; }
        const int nd = nd_of(pb.degree[j]);
        pair_tgt[p] = (int32_t)t;
        pair_patch[p] = (int32_t)j;
        pair_self[p] = self ? 1 : 0;
        pair_off[p] = pos;
        const int64_t nb = pb.node_ptr[j];
        if (col)
            for (int l = 0; l < nd; ++l) col[pos + l] = (int32_t)(nb + l);
        pos += nd;
        ++p;
    }
}

// Scatter pairs into their (degree, kind) segment: slots are counted per
// block in LDS and reserved with one global atomic per (block, key).
__global__ __launch_bounds__(256) void k_group(int64_t np, const int32_t *pair_patch,
                                               const int8_t *pair_self, const int32_t *degree,
                                               const int64_t *seg_start,
                                               unsigned long long *cursor, int32_t *grp)
{
    __shared__ unsigned int s_cnt[18];
    __shared__ unsigned long long s_base[18];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (threadIdx.x < 18) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    int key = -1;
    unsigned int local = 0;
    if (p < np) {
        key = (pair_self[p] ? 9 : 0) + degree[pair_patch[p]];
        local = atomicAdd(&s_cnt[key], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 18 && s_cnt[threadIdx.x] > 0)
        s_base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x], (unsigned long long)s_cnt[threadIdx.x]);
    __syncthreads();
    if (key >= 0) grp[seg_start[key] + (int64_t)(s_base[key] + local)] = (int32_t)p;
}

// ---------------------------------------------------------- patch prep

template <int D>
__device__ void prep_patch(const Problem &pb, const DegTab &tab, int64_t j, double tol_scale,
                           double *coef, double *coef_rel, double *tau, double *rho, int *flags)
{
    constexpr int ND = nd_of(D);
    const double *V = tab.V[D];
    const double *x = pb.xyz + 3 * pb.node_ptr[j];
    double *cf = coef + 3 * pb.node_ptr[j];
    for (int a = 0; a < ND; ++a) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int l = 0; l < ND; ++l) {
            const double v = V[a * ND + l];
            s0 = __builtin_fma(v, x[3 * l + 0], s0);
            s1 = __builtin_fma(v, x[3 * l + 1], s1);
            s2 = __builtin_fma(v, x[3 * l + 2], s2);
        }
        cf[0 * ND + a] = s0;
        cf[1 * ND + a] = s1;
        cf[2 * ND + a] = s2;
        double *cr = coef_rel + 3 * pb.node_ptr[j];
        cr[0 * ND + a] = a == 0 ? 0.0 : s0;
        cr[1 * ND + a] = a == 0 ? 0.0 : s1;
        cr[2 * ND + a] = a == 0 ? 0.0 : s2;
    }
    // d_j = min_l sqrt(J(u_l, v_l) |w_l|)  (Section 4.2)
    double dj = 1e300;
    bool bad = false;
    for (int l = 0; l < ND; ++l) {
        double K[ND], X[3], Xu[3], Xv[3];
        chart_eval<D>(cf, tab.uv[D][2 * l], tab.uv[D][2 * l + 1], K, X, Xu, Xv);
        const double n0 = Xu[1] * Xv[2] - Xu[2] * Xv[1];
        const double n1 = Xu[2] * Xv[0] - Xu[0] * Xv[2];
        const double n2 = Xu[0] * Xv[1] - Xu[1] * Xv[0];
        const double J = __builtin_sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        if (!(J > 0.0) || !(J < 1e300)) bad = true;
        const double q = __builtin_sqrt(J * __builtin_fabs(tab.w[D][l]));
        dj = q < dj ? q : dj;
    }
    if (bad) flags[kFlagDegenerate] = 1;
    tau[j] = tol_scale * dj / tab.normV[D];
    double rh = 0.0;
    for (int l = 0; l < ND; ++l)
        rh = __builtin_fmax(rh, __builtin_sqrt(x[3 * l] * x[3 * l] + x[3 * l + 1] * x[3 * l + 1] +
                                               x[3 * l + 2] * x[3 * l + 2]));
    rho[j] = rh;
}

__global__ void k_prep(Problem pb, DegTab tab, double tol_scale, double *coef, double *coef_rel,
                       double *tau, double *rho, int *flags)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= pb.P) return;
    switch (pb.degree[j]) {
    case 1: prep_patch<1>(pb, tab, j, tol_scale, coef, coef_rel, tau, rho, flags); break;
    case 2: prep_patch<2>(pb, tab, j, tol_scale, coef, coef_rel, tau, rho, flags); break;
    case 3: prep_patch<3>(pb, tab, j, tol_scale, coef, coef_rel, tau, rho, flags); break;
    case 4: prep_patch<4>(pb, tab, j, tol_scale, coef, coef_rel, tau, rho, flags); break;
    case 5: prep_patch<5>(pb, tab, j, tol_scale, coef, coef_rel, tau, rho, flags); break;
    case 6: prep_patch<6>(pb, tab, j, tol_scale, coef, coef_rel, tau, rho, flags); break;
    case 7: prep_patch<7>(pb, tab, j, tol_scale, coef, coef_rel, tau, rho, flags); break;
    case 8: prep_patch<8>(pb, tab, j, tol_scale, coef, coef_rel, tau, rho, flags); break;
    default: flags[kFlagNotRegistered] = 1; break;
    }
}

// ------------------------------------------------------ quadrature args

struct QuadArgs {
    Problem pb;
    DegTab tab;
    Kern kern;
    int helm;
    int max_depth;
    int min_depth;
    const double *rule;   // [64][3] subtriangle rule (u, v, w)
    const double *glr;    // [nr][2] radial Gauss-Legendre (s, w) on [0,1]
    const double *gla;    // [na][2] angular Gauss-Legendre (t, w) on [0,1]
    int nr, na;
    const int32_t *grp;
    int64_t seg, count;   // segment start and length in grp
    const int32_t *pair_tgt, *pair_patch;
    const int64_t *pair_off;
    const double *coef;
    // the same coefficients without the constant term (basis 0): positions
    // relative to it, of the patch's size rather than the surface's, so that
    // x - y near a self target keeps its digits
    const double *coef_rel;
    const double *tau;
    const double *rho;    // max_l |x_l| per patch (coordinate scale)
    double *val;
    double *stack;        // near: [waves][kStack][entry]
    int *flags;
    unsigned long long *stats;
};

template <int D, bool CPLX>
struct QuadShape {
    static constexpr int ND = nd_of(D);
    static constexpr int NV = CPLX ? 2 * ND : ND;  // real components of a moment vector
    static constexpr int NVP = NV | 1;              // odd LDS row pitch
    static constexpr int WPB = (64 * NVP * 8 <= 24 * 1024) ? 4 : 2;  // waves per block
    static constexpr int ESZ = 8 + NV;              // stack entry: tri[6], depth, pad, I[NV]
};

// Reduce per-lane vectors acc[NV] over groups of `G` consecutive lanes into
// out[(lane / G) * NV + v] in LDS (G = 64: whole wave; G = 16: 4 groups).
template <int NV, int NVP, int G>
__device__ __forceinline__ void lds_group_reduce(double *red, double *out, const double *acc,
                                                 int lane)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) red[lane * NVP + v] = acc[v];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    constexpr int NOUT = (64 / G) * NV;
    for (int o = lane; o < NOUT; o += 64) {
        const int g = o / NV, v = o - g * NV;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < G; ++i) s += red[(g * G + i) * NVP + v];
        out[o] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Accumulate f * K into acc (complex f -> interleaved re/im components).
template <int ND, bool CPLX>
__device__ __forceinline__ void acc_products(double *acc, const double *K, double fr, double fi)
{
#pragma unroll
    for (int a = 0; a < ND; ++a) {
        if (CPLX) {
            acc[2 * a] = __builtin_fma(fr, K[a], acc[2 * a]);
            acc[2 * a + 1] = __builtin_fma(fi, K[a], acc[2 * a + 1]);
        } else {
            acc[a] = __builtin_fma(fr, K[a], acc[a]);
        }
    }
}

// ------------------------------------------------ adaptive near quadrature

template <int D, bool CPLX>
__global__ __launch_bounds__((64 * QuadShape<D, CPLX>::WPB)) void k_near(QuadArgs a)
{
    using S = QuadShape<D, CPLX>;
    constexpr int ND = S::ND, NV = S::NV, NVP = S::NVP, WPB = S::WPB, ESZ = S::ESZ;
    constexpr int NL = (NV + 63) / 64;
    __shared__ double s_red[WPB][64 * NVP];
    __shared__ double s_out[WPB][4 * NV];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double *red = s_red[wv];
    double *out = s_out[wv];
    const int64_t wave_id = (int64_t)blockIdx.x * WPB + wv;
    const int64_t nwaves = (int64_t)gridDim.x * WPB;
    double *stk = a.stack + wave_id * (int64_t)kStack * ESZ;
    const int cg = lane >> 4;  // child triangle handled by this lane
    // this lane's rule nodes: root phase node `lane`; child phase nodes
    // (lane & 15) + 16 i, i = 0..3
    const double r_u = a.rule[3 * lane], r_v = a.rule[3 * lane + 1], r_w = a.rule[3 * lane + 2];
    unsigned long long st_visits = 0, st_checks = 0, st_nonconv = 0, st_maxlev = 0, st_pairs = 0;
    int singular = 0, overflow = 0;
    for (int64_t idx = wave_id; idx < a.count; idx += nwaves) {
        const int p = __builtin_amdgcn_readfirstlane(a.grp[a.seg + idx]);
        if (p < 0) continue;
        const int t = __builtin_amdgcn_readfirstlane(a.pair_tgt[p]);
        const int j = __builtin_amdgcn_readfirstlane(a.pair_patch[p]);
        const double *cf = a.coef + 3 * a.pb.node_ptr[j];
        const double x[3] = {a.pb.txyz[3 * (int64_t)t], a.pb.txyz[3 * (int64_t)t + 1],
                             a.pb.txyz[3 * (int64_t)t + 2]};
        const double tau = a.tau[j];
        const double nfac = noise_factor(__builtin_sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) +
                                         a.rho[j]);
        ++st_pairs;
        // root: one node per lane
        double acc[NV];
        {
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = 0.0;
            double K[ND], X[3], Xu[3], Xv[3];
            chart_eval<D>(cf, r_u, r_v, K, X, Xu, Xv);
            const double n[3] = {Xu[1] * Xv[2] - Xu[2] * Xv[1], Xu[2] * Xv[0] - Xu[0] * Xv[2],
                                 Xu[0] * Xv[1] - Xu[1] * Xv[0]};
            double fr, fi;
            kern_eval(a.kern, a.helm, x, X, n, fr, fi, singular);
            acc_products<ND, CPLX>(acc, K, fr * r_w, fi * r_w);
        }
        lds_group_reduce<NV, NVP, 64>(red, out, acc, lane);
        // push root
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int v = lane + 64 * k;
            if (v < NV) stk[8 + v] = out[v];
        }
        if (lane < 8) {
            const double root[8] = {0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0};
            double rv = 0.0;
#pragma unroll
            for (int k = 0; k < 8; ++k) rv = (k == lane) ? root[k] : rv;
            stk[lane] = rv;
        }
        int sp = 1;
        ++st_visits;
        double tot[NL];  // lane owns components lane + 64 k
#pragma unroll
        for (int k = 0; k < NL; ++k) tot[k] = 0.0;
        bool nonconv = false;
        while (sp > 0) {
            --sp;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const double *e = stk + (int64_t)sp * ESZ;
            // entry header read with per-lane vector loads, then broadcast
            const double hv = lane < 8 ? e[lane] : 0.0;
            const double ax = __shfl(hv, 0, 64), ay = __shfl(hv, 1, 64);
            const double bx = __shfl(hv, 2, 64), by = __shfl(hv, 3, 64);
            const double cx = __shfl(hv, 4, 64), cy = __shfl(hv, 5, 64);
            const int depth = (int)__shfl(hv, 6, 64);
            double IT[NL];
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int v = lane + 64 * k;
                IT[k] = v < NV ? e[8 + v] : 0.0;
            }
            // this lane's child triangle (A, B, C)
            const double abx = 0.5 * (ax + bx), aby = 0.5 * (ay + by);
            const double bcx = 0.5 * (bx + cx), bcy = 0.5 * (by + cy);
            const double cax = 0.5 * (cx + ax), cay = 0.5 * (cy + ay);
            double Ax, Ay, Bx, By, Cx, Cy;
            if (cg == 0) { Ax = ax; Ay = ay; Bx = abx; By = aby; Cx = cax; Cy = cay; }
            else if (cg == 1) { Ax = abx; Ay = aby; Bx = bx; By = by; Cx = bcx; Cy = bcy; }
            else if (cg == 2) { Ax = cax; Ay = cay; Bx = bcx; By = bcy; Cx = cx; Cy = cy; }
            else { Ax = bcx; Ay = bcy; Bx = cax; By = cay; Cx = abx; Cy = aby; }
            const double area = __builtin_ldexp(1.0, -2 * (depth + 1));  // |C| / |T0|
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = 0.0;
            double sens = 0.0;
#pragma unroll 1
            for (int i = 0; i < 4; ++i) {
                const int q = (lane & 15) + 16 * i;
                const double ru = a.rule[3 * q], rv = a.rule[3 * q + 1], rw = a.rule[3 * q + 2];
                const double u = Ax + ru * (Bx - Ax) + rv * (Cx - Ax);
                const double v = Ay + ru * (By - Ay) + rv * (Cy - Ay);
                double K[ND], X[3], Xu[3], Xv[3];
                chart_eval<D>(cf, u, v, K, X, Xu, Xv);
                const double n[3] = {Xu[1] * Xv[2] - Xu[2] * Xv[1], Xu[2] * Xv[0] - Xu[0] * Xv[2],
                                     Xu[0] * Xv[1] - Xu[1] * Xv[0]};
                double fr, fi, sn;
                kern_eval(a.kern, a.helm, x, X, n, fr, fi, singular, sn);
                const double w = rw * area;
                acc_products<ND, CPLX>(acc, K, fr * w, fi * w);
                double kk2 = 0.0;
#pragma unroll
                for (int m = 0; m < ND; ++m) kk2 = __builtin_fma(K[m], K[m], kk2);
                sens = __builtin_fma(sn * w * w, kk2, sens);
            }
            const double noise2 = nfac * wave_sum(sens);
            lds_group_reduce<NV, NVP, 16>(red, out, acc, lane);
            // out[c * NV + v] = component v of the moments of child c
            double Sv[NL], e2 = 0.0;
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int v = lane + 64 * k;
                Sv[k] = v < NV ? out[v] + out[NV + v] + out[2 * NV + v] + out[3 * NV + v] : 0.0;
                const double df = Sv[k] - IT[k];
                e2 += df * df;
            }
            const double err2 = wave_sum(e2);
            const double thr = tau * __builtin_ldexp(1.0, -2 * depth);
            st_visits += 4;
            ++st_checks;
            const bool ok = err2 <= thr * thr || err2 <= noise2;
            bool accept = ok && depth + 1 >= a.min_depth;
            if (!accept && (depth + 1 >= a.max_depth || sp + 4 > kStack)) {
                if (sp + 4 > kStack) overflow = 1;
                accept = true;
                if (!ok) nonconv = true;
            }
            if (accept) {
#pragma unroll
                for (int k = 0; k < NL; ++k) tot[k] += Sv[k];
                if ((unsigned long long)(depth + 1) > st_maxlev) st_maxlev = depth + 1;
            } else {
                // push children 3, 2, 1, 0 so that child 0 is processed next
                for (int c = 3; c >= 0; --c) {
                    double *ne = stk + (int64_t)sp * ESZ;
#pragma unroll
                    for (int k = 0; k < NL; ++k) {
                        const int v = lane + 64 * k;
                        if (v < NV) ne[8 + v] = out[c * NV + v];
                    }
                    if (lane < 8) {
                        double tA0, tA1, tB0, tB1, tC0, tC1;
                        if (c == 0) { tA0 = ax; tA1 = ay; tB0 = abx; tB1 = aby; tC0 = cax; tC1 = cay; }
                        else if (c == 1) { tA0 = abx; tA1 = aby; tB0 = bx; tB1 = by; tC0 = bcx; tC1 = bcy; }
                        else if (c == 2) { tA0 = cax; tA1 = cay; tB0 = bcx; tB1 = bcy; tC0 = cx; tC1 = cy; }
                        else { tA0 = bcx; tA1 = bcy; tB0 = cax; tB1 = cay; tC0 = abx; tC1 = aby; }
                        const double hdr[8] = {tA0, tA1, tB0, tB1, tC0, tC1, (double)(depth + 1), 0.0};
                        double hvv = 0.0;
#pragma unroll
                        for (int k = 0; k < 8; ++k) hvv = (k == lane) ? hdr[k] : hvv;
                        ne[lane] = hvv;
                    }
                    ++sp;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        }
        if (nonconv) ++st_nonconv;
        const int64_t off = a.pair_off[p];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int v = lane + 64 * k;
            if (v < NV) a.val[(CPLX ? 2 : 1) * off + v] = tot[k];
        }
    }
    singular = wave_or(singular);
    overflow = wave_or(overflow);
    if (lane == 0) {
        if (singular) a.flags[kFlagSingular] = 1;
        if (overflow) a.flags[kFlagStackOverflow] = 1;
        atomicAdd(&a.stats[kStatNear], st_pairs);
        atomicAdd(&a.stats[kStatVisits], st_visits);
        atomicAdd(&a.stats[kStatChecks], st_checks);
        atomicAdd(&a.stats[kStatNonconv], st_nonconv);
        atomicMax(&a.stats[kStatMaxLevel], st_maxlev);
    }
}

// -------------------------------------------------------- self quadrature

constexpr int kPanW = 9;

template <int D, bool CPLX>
struct SelfShape {
    static constexpr int ND = nd_of(D);
    static constexpr int NV = CPLX ? 2 * ND : ND;
    static constexpr int RP = (ND + 2) | 1;   // LDS row pitch: K[ND], f_re w, f_im w
    static constexpr int WPB = 2;
    // small moment vectors are accumulated per lane in registers and reduced
    // once per target; large ones are staged through LDS every 64 nodes
    static constexpr int W = (NV + 15) / 16 * 16;
    static constexpr bool REG = W <= 32;
};

// 16-lane reduce-scatter: on entry acc[W] holds this lane's partial sums;
// on exit acc[0..W/16) holds components [W/16 (lane & 15), W/16 (lane & 15)
// + W/16) summed over the 16 lanes of the lane's row.
template <int W>
__device__ __forceinline__ void reduce_scatter_rows(double *acc, int lane)
{
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        const int m = 8 >> step;
        const int w = W >> (step + 1);
        const bool hi = (lane & m) != 0;
#pragma unroll
        for (int i = 0; i < w; ++i) {
            const double lo_v = acc[i], hi_v = acc[i + w];
            const double send = hi ? lo_v : hi_v;
            const double keep = hi ? hi_v : lo_v;
            acc[i] = keep + __shfl_xor(send, m, 64);
        }
    }
}

// Self quadrature.  One wavefront per target; the target-split rule's nodes
// are taken 64 at a time (one per lane), and each lane evaluates chart,
// kernel and basis at its node.  Small degrees (moment vector <= 32 doubles)
// accumulate per lane in registers and reduce-scatter over the wavefront
// once per target, at two wavefronts per SIMD; larger degrees stage K and the
// weighted kernel value in LDS, and lane v accumulates component v of the
// moments over the 64 staged nodes.
template <int D, bool CPLX>
__global__ __launch_bounds__((64 * SelfShape<D, CPLX>::WPB))
__attribute__((amdgpu_waves_per_eu(D <= 4 ? 2 : 1))) void k_self(QuadArgs a)
{
    using S = SelfShape<D, CPLX>;
    constexpr int ND = S::ND, NV = S::NV, RP = S::RP, WPB = S::WPB;
    constexpr int NL = (NV + 63) / 64;
    __shared__ double s_stage[WPB][64 * RP];
    // per wavefront: up to 6 panels x (A, E, mu, h/L, det, xi_a, xi_b)
    __shared__ double s_pan[WPB][6][kPanW];
    __shared__ double s_cfw[WPB][3 * ND];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double *stage = s_stage[wv];
    const int64_t wave_id = (int64_t)blockIdx.x * WPB + wv;
    const int64_t nwaves = (int64_t)gridDim.x * WPB;
    const int nr = a.nr, na = a.na;
    unsigned long long st_pairs = 0;
    int singular = 0;
    for (int64_t idx = wave_id; idx < a.count; idx += nwaves) {
        const int p = __builtin_amdgcn_readfirstlane(a.grp[a.seg + idx]);
        if (p < 0) continue;
        const int t = __builtin_amdgcn_readfirstlane(a.pair_tgt[p]);
        const int j = __builtin_amdgcn_readfirstlane(a.pair_patch[p]);
        const int64_t nb = a.pb.node_ptr[j];
        const int l = (int)(a.pb.node_of_target[t] - nb);
        // chart coefficients (relative to the constant term) in LDS, read at
        // every node (kept out of registers)
        for (int k = lane; k < 3 * ND; k += 64) s_cfw[wv][k] = a.coef_rel[3 * nb + k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double *cf = s_cfw[wv];
        const double tu = a.tab.uv[D][2 * l], tv = a.tab.uv[D][2 * l + 1];
        ++st_pairs;
        // target = chart point X(t); first fundamental form at t
        double x[3], G00, G01, G11;
        {
            double K[ND], Xu[3], Xv[3];
            chart_eval<D>(cf, tu, tv, K, x, Xu, Xv);
            G00 = Xu[0] * Xu[0] + Xu[1] * Xu[1] + Xu[2] * Xu[2];
            G01 = Xu[0] * Xv[0] + Xu[1] * Xv[1] + Xu[2] * Xv[2];
            G11 = Xv[0] * Xv[0] + Xv[1] * Xv[1] + Xv[2] * Xv[2];
        }
        // panels: for each edge (P_e, P_e+1) of T0 the triangle (t, P_e, P_e+1)
        // is collapsed at t: y = t + s (A + lam E - t).  In the metric G the
        // distance from t to the edge point is sqrt(h^2 + (lam - mu)^2 L^2);
        // lam = mu + (h/L) sinh(xi) makes the angular integrand smooth.  The
        // panel is split at the foot (xi = 0) when it lies inside the edge.
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
                // the values are uniform over the wavefront: one lane stores them
                if (lane == 0) {
                    double *pp = s_pan[wv][npan];
                    pp[0] = Ax; pp[1] = Ay; pp[2] = Ex; pp[3] = Ey;
                    pp[4] = mu; pp[5] = h / L; pp[6] = det;
                    pp[7] = split ? (half == 0 ? x0 : 0.0) : x0;
                    pp[8] = split ? (half == 0 ? 0.0 : x1) : x1;
                }
                ++npan;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int per_panel = na * nr;
        const int total = npan * per_panel;
        // node q -> panel, angular, radial index (float reciprocals: exact
        // for these small integers)
        const float inv_pp = 1.0f / (float)per_panel, inv_nr = 1.0f / (float)nr;
        if constexpr (S::REG) {
            constexpr int W = S::W, PL = W / 16;
            double racc[W];
#pragma unroll
            for (int v = 0; v < W; ++v) racc[v] = 0.0;
            for (int q = lane; q < total; q += 64) {
                const int pi = (int)(((float)q + 0.5f) * inv_pp);
                const int rem = q - pi * per_panel;
                const int ia = (int)(((float)rem + 0.5f) * inv_nr), ir = rem - ia * nr;
                const double *pp = s_pan[wv][pi];
                const double Ax = pp[0], Ay = pp[1], Ex = pp[2], Ey = pp[3], mu = pp[4];
                const double hl = pp[5], det = pp[6], xa = pp[7], xb = pp[8];
                const double xi = xa + (xb - xa) * a.gla[2 * ia];
                // sinh and cosh from one exponential (lam needs absolute accuracy)
                const double ex = exp(xi), exi = 1.0 / ex;
                const double lam = mu + hl * (0.5 * (ex - exi));
                const double dlam = hl * (0.5 * (ex + exi)) * (xb - xa) * a.gla[2 * ia + 1];
                const double s = a.glr[2 * ir], ws = a.glr[2 * ir + 1];
                const double dx = Ax + lam * Ex - tu, dy = Ay + lam * Ey - tv;
                double K[ND], X[3], Xu[3], Xv[3];
                const double *cfn = cf;
                asm volatile("" : "+v"(cfn));
                chart_eval<D>(cfn, tu + s * dx, tv + s * dy, K, X, Xu, Xv);
                const double n[3] = {Xu[1] * Xv[2] - Xu[2] * Xv[1], Xu[2] * Xv[0] - Xu[0] * Xv[2],
                                     Xu[0] * Xv[1] - Xu[1] * Xv[0]};
                double fr, fi;
                kern_eval(a.kern, a.helm, x, X, n, fr, fi, singular);
                const double w = s * det * ws * dlam;
                fr *= w;
                fi *= w;
#pragma unroll
                for (int m = 0; m < ND; ++m) {
                    if (CPLX) {
                        racc[2 * m] = __builtin_fma(fr, K[m], racc[2 * m]);
                        racc[2 * m + 1] = __builtin_fma(fi, K[m], racc[2 * m + 1]);
                    } else {
                        racc[m] = __builtin_fma(fr, K[m], racc[m]);
                    }
                }
            }
            reduce_scatter_rows<W>(racc, lane);
#pragma unroll
            for (int i = 0; i < PL; ++i) {
                racc[i] += __shfl_xor(racc[i], 16, 64);
                racc[i] += __shfl_xor(racc[i], 32, 64);
            }
            if (lane < 16) {
                const int64_t off = a.pair_off[p];
#pragma unroll
                for (int i = 0; i < PL; ++i) {
                    const int v = PL * lane + i;
                    if (v < NV) a.val[(CPLX ? 2 : 1) * off + v] = racc[i];
                }
            }
            continue;
        }
        double acc[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) acc[k] = 0.0;
        for (int base = 0; base < total; base += 64) {
            const int q = base + lane;
            double fr = 0.0, fi = 0.0;
            double K[ND];
#pragma unroll
            for (int m = 0; m < ND; ++m) K[m] = 0.0;
            if (q < total) {
                const int pi = (int)(((float)q + 0.5f) * inv_pp);
                const int rem = q - pi * per_panel;
                const int ia = (int)(((float)rem + 0.5f) * inv_nr), ir = rem - ia * nr;
                const double *pp = s_pan[wv][pi];
                const double Ax = pp[0], Ay = pp[1], Ex = pp[2], Ey = pp[3], mu = pp[4];
                const double hl = pp[5], det = pp[6], xa = pp[7], xb = pp[8];
                const double xi = xa + (xb - xa) * a.gla[2 * ia];
                // sinh and cosh from one exponential (lam needs absolute accuracy)
                const double ex = exp(xi), exi = 1.0 / ex;
                const double lam = mu + hl * (0.5 * (ex - exi));
                const double dlam = hl * (0.5 * (ex + exi)) * (xb - xa) * a.gla[2 * ia + 1];
                const double s = a.glr[2 * ir], ws = a.glr[2 * ir + 1];
                const double dx = Ax + lam * Ex - tu, dy = Ay + lam * Ey - tv;
                double X[3], Xu[3], Xv[3];
                chart_eval<D>(cf, tu + s * dx, tv + s * dy, K, X, Xu, Xv);
                const double n[3] = {Xu[1] * Xv[2] - Xu[2] * Xv[1], Xu[2] * Xv[0] - Xu[0] * Xv[2],
                                     Xu[0] * Xv[1] - Xu[1] * Xv[0]};
                kern_eval(a.kern, a.helm, x, X, n, fr, fi, singular);
                const double w = s * det * ws * dlam;
                fr *= w;
                fi *= w;
            }
            double *row = stage + lane * RP;
#pragma unroll
            for (int m = 0; m < ND; ++m) row[m] = K[m];
            row[ND] = fr;
            row[ND + 1] = fi;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int v = lane + 64 * k;
                if (v < NV) {
                    const int m = CPLX ? (v >> 1) : v;
                    const int part = CPLX ? (v & 1) : 0;
                    double sacc = acc[k];
                    for (int i = 0; i < 64; ++i)
                        sacc = __builtin_fma(stage[i * RP + ND + part], stage[i * RP + m], sacc);
                    acc[k] = sacc;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        const int64_t off = a.pair_off[p];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int v = lane + 64 * k;
            if (v < NV) a.val[(CPLX ? 2 : 1) * off + v] = acc[k];
        }
    }
    singular = wave_or(singular);
    if (lane == 0) {
        if (singular) a.flags[kFlagSingular] = 1;
        atomicAdd(&a.stats[kStatSelf], st_pairs);
    }
}

// ------------------------------------------- moments -> node weights

typedef double v4f64 __attribute__((ext_vector_type(4)));

template <int D, bool CPLX>
struct WeightsShape {
    static constexpr int ND = nd_of(D);
    static constexpr int C = CPLX ? 2 : 1;
    static constexpr int PPT = 16 / C;          // pairs per 16-row tile
    static constexpr int KS = (ND + 3) / 4;     // k steps of the 16x16x4 product
    static constexpr int NTL = (ND + 15) / 16;  // 16-column tiles
};

// Moments -> node weights, in place on the output blocks of a (degree, kind)
// segment: a_l = sum_nm V_(nm),l I_nm (Section 4.3), as a batched product on
// the FP64 matrix cores.  Rows are (pair, re/im), columns the node l, the
// contraction runs over the basis index:  A[row][m] = I_m, B[m][l] = V_(m),l.
// One wavefront per 16 rows (8 complex or 16 real pairs).  Operand layout of
// the 16x16x4 f64 product: lane q holds A[q % 16][q / 16], B[q / 16][q % 16]
// and D[q / 16 + 4 r][q % 16], r = 0..3.  Each wavefront reads all moments of
// its pairs before it writes their weights.
template <int D, bool CPLX>
__global__ __launch_bounds__(256) void k_weights(const int32_t *grp, int64_t seg, int64_t count,
                                                 const int64_t *pair_off, const double *V,
                                                 double *val)
{
    using S = WeightsShape<D, CPLX>;
    constexpr int ND = S::ND, C = S::C, PPT = S::PPT, KS = S::KS, NTL = S::NTL;
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t ntiles = (count + PPT - 1) / PPT;
    if (tile >= ntiles) return;  // uniform over the wavefront
    // the A row of this lane
    const int ia = lane & 15;
    const int64_t ipa = tile * PPT + ia / C;
    const int pa = ipa < count ? grp[seg + ipa] : -1;
    const int64_t offa = pa >= 0 ? pair_off[pa] : -1;
    const int parta = ia % C;
    v4f64 acc[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[t] = v4f64{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int m = 4 * s + (lane >> 4);
        const double av = (offa >= 0 && m < ND) ? val[C * (offa + m) + parta] : 0.0;
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
            const int l = 16 * t + (lane & 15);
            const double bv = (m < ND && l < ND) ? V[m * ND + l] : 0.0;
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = (lane >> 4) + 4 * r;
        const int64_t ip = tile * PPT + i / C;
        const int p = ip < count ? grp[seg + ip] : -1;
        if (p < 0) continue;
        const int64_t off = pair_off[p];
#pragma unroll
        for (int t = 0; t < NTL; ++t) {
            const int l = 16 * t + (lane & 15);
            if (l < ND) val[C * (off + l) + i % C] = acc[t][r];
        }
    }
}

// -------------------------------------------------------------- apply

template <bool CPLX>
__global__ __launch_bounds__(256) void k_apply(int64_t NT, const int64_t *row_ptr,
                                               const int32_t *col, const double *val,
                                               const double *sigma, double *y)
{
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= NT) return;
    double sr = 0.0, si = 0.0;
    for (int64_t e = row_ptr[row] + lane; e < row_ptr[row + 1]; e += 64) {
        const int64_t c = col[e];
        if (CPLX) {
            const double ar = val[2 * e], ai = val[2 * e + 1];
            const double gr = sigma[2 * c], gi = sigma[2 * c + 1];
            sr += ar * gr - ai * gi;
            si += ar * gi + ai * gr;
        } else {
            sr += val[e] * sigma[c];
        }
    }
    sr = wave_sum(sr);
    if (CPLX) si = wave_sum(si);
    if (lane == 0) {
        if (CPLX) { y[2 * row] = sr; y[2 * row + 1] = si; }
        else y[row] = sr;
    }
}

}  // namespace nfq
