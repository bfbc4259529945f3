// nfq_api.hip -- C ABI of the near-field correction generator (include/nfq.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nfq.h"
#include "kernels.hpp"
#include "near_patch.hpp"
#include "nearlist.hpp"
#include "adjoint.hpp"
#include "tables.hpp"

using namespace nfq;

struct nfq_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    RefData ref[9];
    double *dV[9] = {}, *duv[9] = {}, *dw[9] = {}, *dD[9] = {};
    double *drule = nullptr;         // [64][3]
    double *dgl = nullptr;   // Gauss-Legendre rules 1..64 on [0,1]
    std::string err;
};

struct nfq_plan {
    nfq_ctx *ctx = nullptr;
    int device = 0;   // kept here so that destroying a plan never reads its context
    Problem pb{};
    int64_t nnz = 0, npairs = 0;
    int64_t *row_ptr = nullptr;      // caller's
    // scratch
    int64_t *rowlen = nullptr, *npair = nullptr, *pair_ptr = nullptr;
    std::vector<int64_t *> scan_tmp; // per level: a_tot, b_tot, a_off, b_off
    std::vector<int64_t> scan_n;
    int32_t *pair_tgt = nullptr, *pair_patch = nullptr;
    int8_t *pair_self = nullptr;
    int64_t *pair_off = nullptr;
    int32_t *grp = nullptr;
    int64_t grp_len = 0;
    int64_t seg_start_h[18] = {}, seg_len_h[18] = {}, count_h[18] = {};
    int64_t *seg_start = nullptr;
    unsigned long long *cursor = nullptr;
    double *coef = nullptr, *coef_rel = nullptr, *tau = nullptr, *rho = nullptr;
    double *stack = nullptr;
    int64_t stack_waves = 0;
    int *flags = nullptr;
    unsigned long long *stats = nullptr;
    unsigned long long *counts = nullptr;
    int present_mask = 0;
    int max_degree = 0;
    int value_kind = -1;  // value type of the last generate: 0 double, 1 complex128
    // patch-centric near work items
    std::vector<int64_t *> scan_tmp_p;  // scan temporaries for P-sized arrays
    int64_t n_near = 0;
    int64_t *pcount = nullptr, *nchunk = nullptr, *pptr = nullptr, *cptr = nullptr;
    unsigned long long *pcursor = nullptr;
    int32_t *plist = nullptr, *plist_raw = nullptr;
    int32_t *items = nullptr;
    int64_t item_start_h[9] = {}, item_count_h[9] = {}, n_items = 0;
    int64_t *item_start = nullptr;
    unsigned long long *item_cursor = nullptr;
    double *mom = nullptr;
    int64_t mom_slots = 0, mom_slot = 0;
    // adjoint scratch
    double *scoef = nullptr, *gc_item = nullptr, *t_pair = nullptr, *gc_self = nullptr;
    unsigned int *self_mark = nullptr;
    int gc_pitch = 0;
    hipEvent_t ev[2 * 5 * 9] = {};  // phase timing events (begin, end) x phase x degree
    bool ev_ok = false;
};

enum Phase { kPhBuilder = 0, kPhPrep, kPhSelf, kPhNear, kPhWeights, kNumPhases };

struct Timer {
    nfq_plan *pl;
    bool on;
    int used[kNumPhases * 9] = {};
    void begin(int ph, int slot, hipStream_t st)
    {
        if (on) { (void)hipEventRecord(pl->ev[2 * (ph * 9 + slot)], st); used[ph * 9 + slot] = 1; }
    }
    void end(int ph, int slot, hipStream_t st)
    {
        if (on) (void)hipEventRecord(pl->ev[2 * (ph * 9 + slot) + 1], st);
    }
    double total(int ph)
    {
        double t = 0.0;
        for (int s = 0; s < 9; ++s)
            if (used[ph * 9 + s]) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, pl->ev[2 * (ph * 9 + s)], pl->ev[2 * (ph * 9 + s) + 1]) == hipSuccess)
                    t += ms;
            }
        return t;
    }
};

namespace {

thread_local std::string g_err;  // last error of a call that has no context

nfq_status fail(nfq_ctx *ctx, nfq_status s, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    else g_err = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), NFQ_ERR_HIP, std::string(#expr " -> ") + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t n)
{
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

int64_t pad16(int64_t n) { return (n + 15) / 16 * 16; }

// Fill `bytes` (a multiple of 4) at p with the 32-bit word v, as a kernel.
void fill32(void *p, int64_t bytes, uint32_t v, hipStream_t st)
{
    const int64_t n = bytes / 4;
    if (n <= 0) return;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill32, dim3(blocks), dim3(256), 0, st, n, v, (uint32_t *)p);
}

// Exclusive scan of a_in, b_in (length n) into a_out, b_out (length n + 1).
nfq_status run_scan(nfq_ctx *ctx, int64_t n, const int64_t *a_in, const int64_t *b_in,
                    int64_t *a_out, int64_t *b_out, std::vector<int64_t *> &tmp)
{
    hipStream_t st = ctx->stream;
    // level sizes
    std::vector<int64_t> sizes;
    int64_t m = n;
    while (true) {
        sizes.push_back(m);
        if (m <= kScanTile) break;
        m = (m + kScanTile - 1) / kScanTile;
    }
    // level 0 scans the input; level k scans the tile totals of level k-1
    const int64_t *ia = a_in, *ib = b_in;
    int64_t *oa = a_out, *ob = b_out;
    std::vector<int64_t *> outs_a, outs_b;
    for (size_t lv = 0; lv < sizes.size(); ++lv) {
        const int64_t len = sizes[lv];
        const int64_t tiles = (len + kScanTile - 1) / kScanTile;
        int64_t *ta = tmp[4 * lv + 0], *tb = tmp[4 * lv + 1];
        int64_t *na = tmp[4 * lv + 2], *nb2 = tmp[4 * lv + 3];
        if (len > 0)
            hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)tiles), dim3(kScanBlock), 0, st, len, ia,
                               ib, oa, ob, ta, tb);
        outs_a.push_back(oa);
        outs_b.push_back(ob);
        ia = ta;
        ib = tb;
        oa = na;
        ob = nb2;
    }
    // propagate tile offsets downwards
    for (int lv = (int)sizes.size() - 2; lv >= 0; --lv) {
        const int64_t len = sizes[lv];
        hipLaunchKernelGGL(k_scan_add, dim3(nblk(len, 256)), dim3(256), 0, st, len, outs_a[lv],
                           outs_b[lv], outs_a[lv + 1], outs_b[lv + 1]);
    }
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, st, n, a_in, b_in, a_out, b_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, NFQ_ERR_HIP, hipGetErrorString(e));
    return NFQ_OK;
}

hipError_t alloc_scan_tmp(int64_t n, std::vector<int64_t *> &tmp)
{
    int64_t m = n;
    while (true) {
        const int64_t tiles = (m + kScanTile - 1) / kScanTile;
        for (int k = 0; k < 4; ++k) {
            int64_t *p = nullptr;
            hipError_t e = dalloc(&p, tiles + 1);
            if (e != hipSuccess) return e;
            tmp.push_back(p);
        }
        if (m <= kScanTile) break;
        m = tiles;
    }
    return hipSuccess;
}

// Per-degree count of work items (chunks of <= 64 near targets of a patch).
__global__ void k_item_count(int64_t P, const int32_t *degree, const int64_t *nchunk,
                             unsigned long long *cnt)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P || nchunk[j] == 0) return;
    atomicAdd(&cnt[degree[j]], (unsigned long long)nchunk[j]);
}

// Patch-major near pairs and work items (generate-time builder part).
nfq_status build_items(nfq_plan *pl, hipStream_t st)
{
    nfq_ctx *ctx = pl->ctx;
    const int64_t P = pl->pb.P, np = pl->npairs;
    fill32(pl->pcount, P * 8, 0u, st);
    fill32(pl->pcursor, P * 8, 0u, st);
    fill32(pl->item_cursor, 9 * 8, 0u, st);
    if (np > 0)
        hipLaunchKernelGGL(k_patch_count, dim3(nblk(np, 256)), dim3(256), 0, st, np, pl->pair_patch,
                           pl->pair_self, pl->pcount);
    hipLaunchKernelGGL(k_patch_chunks, dim3(nblk(P, 256)), dim3(256), 0, st, P, pl->pcount, pl->nchunk);
    nfq_status s = run_scan(pl->ctx, P, pl->pcount, pl->nchunk, pl->pptr, pl->cptr, pl->scan_tmp_p);
    if (s != NFQ_OK) return s;
    if (np > 0)
        hipLaunchKernelGGL(k_patch_scatter, dim3(nblk(np, 256)), dim3(256), 0, st, np, pl->pair_patch,
                           pl->pair_self, pl->pptr, pl->pcursor, pl->plist_raw);
    if (np > 0)
        hipLaunchKernelGGL(k_patch_sort, dim3((unsigned)std::min<int64_t>(std::max<int64_t>(P, 1), 65535)),
                           dim3(256), 0, st, P, pl->pptr, pl->pcount, pl->plist_raw, pl->plist);
    hipLaunchKernelGGL(k_items, dim3(nblk(P, 256)), dim3(256), 0, st, P, pl->pb.degree, pl->pcount,
                       pl->pptr, pl->item_start, pl->item_cursor, pl->items);
    HIP_TRY(ctx, hipGetLastError());
    return NFQ_OK;
}

DegTab make_tab(const nfq_ctx *ctx)
{
    DegTab t{};
    for (int d = 0; d < 9; ++d) {
        t.V[d] = ctx->dV[d];
        t.uv[d] = ctx->duv[d];
        t.w[d] = ctx->dw[d];
        t.D[d] = ctx->dD[d];
        t.normV[d] = ctx->ref[d].normV;
        t.present[d] = ctx->dV[d] != nullptr;
    }
    return t;
}

nfq_status check_flags(nfq_ctx *ctx, const int *hflags)
{
    if (hflags[kFlagInvalid]) return fail(ctx, NFQ_ERR_INVALID_ARG, "invalid near list or node id");
    if (hflags[kFlagNotRegistered])
        return fail(ctx, NFQ_ERR_NOT_REGISTERED, "a patch uses an unregistered degree");
    if (hflags[kFlagDegenerate]) return fail(ctx, NFQ_ERR_DEGENERATE_PATCH, "degenerate patch (J <= 0)");
    if (hflags[kFlagSingular])
        return fail(ctx, NFQ_ERR_SINGULAR_PAIR, "a near target coincides with a patch point");
    return NFQ_OK;
}

template <int D, bool CPLX>
void launch_quad(const nfq_plan *pl, QuadArgs qa, int64_t near_seg, int64_t near_cnt,
                 int64_t self_seg, int64_t self_cnt, hipStream_t st, Timer &tm, bool per_pair,
                 PatchArgs pa)
{
    using S = QuadShape<D, CPLX>;
    if (self_cnt > 0) {
        qa.seg = self_seg;
        qa.count = self_cnt;
        using SS = SelfShape<D, CPLX>;
        const unsigned blocks = nblk(self_cnt, SS::WPB);
        tm.begin(kPhSelf, D, st);
        hipLaunchKernelGGL((k_self<D, CPLX>), dim3(blocks), dim3(64 * SS::WPB), 0, st, qa);
        tm.end(kPhSelf, D, st);
    }
    if (near_cnt > 0 && per_pair) {
        qa.seg = near_seg;
        qa.count = near_cnt;
        const int64_t max_blocks = pl->stack_waves / S::WPB;
        const unsigned blocks = (unsigned)std::min<int64_t>(nblk(near_cnt, S::WPB), max_blocks);
        tm.begin(kPhNear, D, st);
        hipLaunchKernelGGL((k_near<D, CPLX>), dim3(blocks), dim3(64 * S::WPB), 0, st, qa);
        tm.end(kPhNear, D, st);
    } else if (pl->item_count_h[D] > 0) {
        pa.item_seg = pl->item_start_h[D];
        pa.item_count = pl->item_count_h[D];
        const unsigned blocks = (unsigned)std::min<int64_t>(pa.item_count, pl->mom_slots);
        tm.begin(kPhNear, D, st);
        hipLaunchKernelGGL((k_near_patch<D, CPLX>), dim3(blocks), dim3(256), 0, st, pa);
        tm.end(kPhNear, D, st);
    }
    const int64_t tot = near_cnt + self_cnt;  // both padded to 16, contiguous
    if (tot > 0) {
        tm.begin(kPhWeights, D, st);
        using WS = WeightsShape<D, CPLX>;
        const int64_t tiles = (tot + WS::PPT - 1) / WS::PPT;  // 16-row tiles, 4 per block
        hipLaunchKernelGGL((k_weights<D, CPLX>), dim3(nblk(tiles, 4)), dim3(256), 0, st, qa.grp,
                           near_seg, tot, qa.pair_off, pl->ctx->dV[D], qa.val);
        tm.end(kPhWeights, D, st);
    }
}

template <bool CPLX>
void launch_degree(int d, const nfq_plan *pl, const QuadArgs &qa, int64_t ns, int64_t nc,
                   int64_t ss, int64_t sc, hipStream_t st, Timer &tm, bool pp, const PatchArgs &pa)
{
    switch (d) {
    case 1: launch_quad<1, CPLX>(pl, qa, ns, nc, ss, sc, st, tm, pp, pa); break;
    case 2: launch_quad<2, CPLX>(pl, qa, ns, nc, ss, sc, st, tm, pp, pa); break;
    case 3: launch_quad<3, CPLX>(pl, qa, ns, nc, ss, sc, st, tm, pp, pa); break;
    case 4: launch_quad<4, CPLX>(pl, qa, ns, nc, ss, sc, st, tm, pp, pa); break;
    case 5: launch_quad<5, CPLX>(pl, qa, ns, nc, ss, sc, st, tm, pp, pa); break;
    case 6: launch_quad<6, CPLX>(pl, qa, ns, nc, ss, sc, st, tm, pp, pa); break;
    case 7: launch_quad<7, CPLX>(pl, qa, ns, nc, ss, sc, st, tm, pp, pa); break;
    case 8: launch_quad<8, CPLX>(pl, qa, ns, nc, ss, sc, st, tm, pp, pa); break;
    default: break;
    }
}

// Gauss-Legendre rules on [0,1] with n = 1..kMaxGL points, rule n at pairs
// [n (n - 1) / 2, n (n + 1) / 2) of ctx->dgl as (node, weight).
constexpr int kMaxGL = 64;
inline int64_t gl_offset(int n) { return (int64_t)n * (n - 1); }  // in doubles

nfq_status upload_gauss_rules(nfq_ctx *ctx)
{
    std::vector<double> buf((size_t)kMaxGL * (kMaxGL + 1)), x, w;
    for (int n = 1; n <= kMaxGL; ++n) {
        gauss_rule(n, 0, 0, x, w);
        for (int i = 0; i < n; ++i) {
            buf[gl_offset(n) + 2 * i] = x[i];
            buf[gl_offset(n) + 2 * i + 1] = w[i];
        }
    }
    HIP_TRY(ctx, dalloc(&ctx->dgl, buf.size()));
    HIP_TRY(ctx, hipMemcpy(ctx->dgl, buf.data(), buf.size() * 8, hipMemcpyHostToDevice));
    return NFQ_OK;
}

// Radial x angular sizes of the self rule per degree (Gauss-Legendre points
// per panel), unless the caller sets them: chosen so that the dual-norm
// error of the self blocks stays well below the tolerance on strongly
// curved mixed-degree surfaces as well as on the spheres.
constexpr int kSelfNr[9] = {10, 10, 10, 10, 14, 16, 18, 18, 20};
constexpr int kSelfNa[9] = {16, 16, 16, 16, 20, 24, 28, 28, 32};

void set_self_rule(const nfq_ctx *ctx, const nfq_params *prm, int d, QuadArgs &qa)
{
    qa.nr = prm->self_nr > 0 ? prm->self_nr : kSelfNr[d];
    qa.na = prm->self_na > 0 ? prm->self_na : kSelfNa[d];
    qa.glr = ctx->dgl + gl_offset(qa.nr);
    qa.gla = ctx->dgl + gl_offset(qa.na);
}

}  // namespace

// Builder, patch preparation and kernel arguments shared by generate and
// adjoint.  col may be null (no column indices written).
static nfq_status prepare(nfq_plan *pl, const nfq_kernel *kern, const nfq_params *prm, int32_t *col,
                   void *val, Timer &tm, bool per_pair, QuadArgs &qa, PatchArgs &pa)
{
    nfq_ctx *ctx = pl->ctx;
    hipStream_t st = ctx->stream;
    const Problem &pb = pl->pb;
    const int64_t NT = pb.NT;
    fill32(pl->flags, kNumFlags * sizeof(int), 0u, st);
    fill32(pl->stats, kNumStats * 8, 0u, st);
    fill32(pl->cursor, 18 * 8, 0u, st);
    fill32(pl->grp, pl->grp_len * sizeof(int32_t), 0xffffffffu, st);
    // pair / work-queue builder
    tm.begin(kPhBuilder, 0, st);
    if (NT > 0)
        hipLaunchKernelGGL(k_rowlen, dim3(nblk(NT, 256)), dim3(256), 0, st, pb, pl->present_mask,
                           pl->rowlen, pl->npair, (unsigned long long *)nullptr, pl->flags);
    nfq_status s = run_scan(pl->ctx, NT, pl->rowlen, pl->npair, pl->row_ptr, pl->pair_ptr, pl->scan_tmp);
    if (s != NFQ_OK) return s;
    if (NT > 0)
        hipLaunchKernelGGL(k_pairs, dim3(nblk(NT, 256)), dim3(256), 0, st, pb, pl->row_ptr,
                           pl->pair_ptr, pl->pair_tgt, pl->pair_patch, pl->pair_self, pl->pair_off,
                           col);
    if (pl->npairs > 0)
        hipLaunchKernelGGL(k_group, dim3(nblk(pl->npairs, 256)), dim3(256), 0, st, pl->npairs,
                           pl->pair_patch, pl->pair_self, pb.degree, pl->seg_start, pl->cursor,
                           pl->grp);
    if (!per_pair) {
        nfq_status sb = build_items(pl, st);
        if (sb != NFQ_OK) return sb;
    }
    tm.end(kPhBuilder, 0, st);
    // patch preparation
    DegTab tab = make_tab(ctx);
    tm.begin(kPhPrep, 0, st);
    hipLaunchKernelGGL(k_prep, dim3(nblk(pb.P, 64)), dim3(64), 0, st, pb, tab,
                       prm->loosen * prm->tol, pl->coef, pl->coef_rel, pl->tau, pl->rho, pl->flags);
    tm.end(kPhPrep, 0, st);
    // quadratures and weights, per degree
    qa.pb = pb;
    qa.tab = tab;
    qa.kern = Kern{kern->alpha_re, kern->alpha_im, kern->beta_re, kern->beta_im, kern->k_re, kern->k_im,
                   std::hypot(kern->beta_re, kern->beta_im)};
    qa.helm = (kern->k_re != 0.0 || kern->k_im != 0.0) ? 1 : 0;
    qa.max_depth = prm->max_depth;
    qa.min_depth = prm->min_depth;
    qa.rule = ctx->drule;
    qa.grp = pl->grp;
    qa.pair_tgt = pl->pair_tgt;
    qa.pair_patch = pl->pair_patch;
    qa.pair_off = pl->pair_off;
    qa.coef = pl->coef;
    qa.coef_rel = pl->coef_rel;
    qa.tau = pl->tau;
    qa.rho = pl->rho;
    qa.val = (double *)val;
    qa.stack = pl->stack;
    qa.flags = pl->flags;
    qa.stats = pl->stats;
    if (!per_pair) {
        // per-slot moment storage of the patch kernel: [max_depth + 1][4][64][W]
        const int64_t wmax = patch_w(pl->max_degree, true);
        const int64_t need = (int64_t)(prm->max_depth + 1) * 4 * 64 * wmax;
        if (need > pl->mom_slot || !pl->mom) {
            if (pl->mom) (void)hipFree(pl->mom);
            pl->mom = nullptr;
            int ncu = 0;
            HIP_TRY(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
            pl->mom_slots = (int64_t)std::max(ncu, 1) * 2;
            HIP_TRY(ctx, dalloc(&pl->mom, pl->mom_slots * need));
            pl->mom_slot = need;
        }
        pa.pb = pb;
        pa.tab = tab;
        pa.kern = qa.kern;
        pa.helm = qa.helm;
        pa.max_depth = prm->max_depth;
        pa.min_depth = prm->min_depth;
        pa.rule = ctx->drule;
        pa.items = pl->items;
        pa.plist = pl->plist;
        pa.pair_tgt = pl->pair_tgt;
        pa.pair_off = pl->pair_off;
        pa.coef = pl->coef;
        pa.tau = pl->tau;
        pa.rho = pl->rho;
        pa.val = (double *)val;
        pa.mom = pl->mom;
        pa.mom_slot = pl->mom_slot;
        pa.flags = pl->flags;
        pa.stats = pl->stats;
    }
    return NFQ_OK;
}

extern "C" {

const char *nfq_status_str(nfq_status s)
{
    switch (s) {
    case NFQ_OK: return "NFQ_OK";
    case NFQ_WARN_NONCONVERGED: return "NFQ_WARN_NONCONVERGED";
    case NFQ_ERR_INVALID_ARG: return "NFQ_ERR_INVALID_ARG";
    case NFQ_ERR_NOT_REGISTERED: return "NFQ_ERR_NOT_REGISTERED";
    case NFQ_ERR_DEGENERATE_PATCH: return "NFQ_ERR_DEGENERATE_PATCH";
    case NFQ_ERR_SINGULAR_PAIR: return "NFQ_ERR_SINGULAR_PAIR";
    case NFQ_ERR_OUT_OF_MEMORY: return "NFQ_ERR_OUT_OF_MEMORY";
    case NFQ_ERR_HIP: return "NFQ_ERR_HIP";
    case NFQ_ERR_UNSUPPORTED: return "NFQ_ERR_UNSUPPORTED";
    default: return "NFQ_UNKNOWN";
    }
}

const char *nfq_last_error(nfq_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

nfq_status nfq_create(int device, void *hip_stream, nfq_ctx **out)
{
    if (!out) return fail(nullptr, NFQ_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    nfq_ctx *ctx = new (std::nothrow) nfq_ctx;
    if (!ctx) return fail(nullptr, NFQ_ERR_OUT_OF_MEMORY, "context");
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    auto bail = [&](nfq_status s, const std::string &m) {
        nfq_destroy(ctx);
        return fail(nullptr, s, m);
    };
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return bail(NFQ_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
    std::vector<double> rule;
    conical_rule(kNG, rule);
    e = dalloc(&ctx->drule, rule.size());
    if (e == hipSuccess) e = hipMemcpy(ctx->drule, rule.data(), rule.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(NFQ_ERR_HIP, std::string("rule upload: ") + hipGetErrorString(e));
    if (upload_gauss_rules(ctx) != NFQ_OK) return bail(NFQ_ERR_HIP, "rule upload: " + ctx->err);
    *out = ctx;
    return NFQ_OK;
}

void nfq_destroy(nfq_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    for (int d = 0; d < 9; ++d) {
        if (ctx->dV[d]) (void)hipFree(ctx->dV[d]);
        if (ctx->duv[d]) (void)hipFree(ctx->duv[d]);
        if (ctx->dw[d]) (void)hipFree(ctx->dw[d]);
        if (ctx->dD[d]) (void)hipFree(ctx->dD[d]);
    }
    if (ctx->drule) (void)hipFree(ctx->drule);
    if (ctx->dgl) (void)hipFree(ctx->dgl);
    delete ctx;
}

nfq_status nfq_register_degree(nfq_ctx *ctx, int d, const double *ref_uv, const double *ref_w)
{
    if (!ctx || !ref_uv) return fail(ctx, NFQ_ERR_INVALID_ARG, "null argument");
    if (d < 1 || d > 8) return fail(ctx, NFQ_ERR_UNSUPPORTED, "degree outside 1..8");
    RefData r;
    std::string msg = build_reference(d, ref_uv, ref_w, r);
    if (!msg.empty()) return fail(ctx, NFQ_ERR_INVALID_ARG, msg);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (ctx->dV[d]) {
        (void)hipFree(ctx->dV[d]); (void)hipFree(ctx->duv[d]); (void)hipFree(ctx->dw[d]);
        (void)hipFree(ctx->dD[d]);
    }
    ctx->dV[d] = ctx->duv[d] = ctx->dw[d] = ctx->dD[d] = nullptr;
    HIP_TRY(ctx, dalloc(&ctx->dV[d], r.V.size()));
    HIP_TRY(ctx, dalloc(&ctx->duv[d], r.uv.size()));
    HIP_TRY(ctx, dalloc(&ctx->dw[d], r.w.size()));
    HIP_TRY(ctx, dalloc(&ctx->dD[d], r.D.size()));
    HIP_TRY(ctx, hipMemcpy(ctx->dV[d], r.V.data(), r.V.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(ctx->duv[d], r.uv.data(), r.uv.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(ctx->dw[d], r.w.data(), r.w.size() * 8, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(ctx->dD[d], r.D.data(), r.D.size() * 8, hipMemcpyHostToDevice));
    ctx->ref[d] = r;
    return NFQ_OK;
}

void nfq_plan_destroy(nfq_plan *pl)
{
    if (!pl) return;
    (void)hipSetDevice(pl->device);
    void *ptrs[] = {pl->rowlen, pl->npair, pl->pair_ptr, pl->pair_tgt, pl->pair_patch, pl->pair_self,
                    pl->pair_off, pl->grp, pl->seg_start, pl->cursor, pl->coef, pl->coef_rel, pl->tau, pl->rho, pl->stack,
                    pl->flags, pl->stats, pl->counts};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int64_t *p : pl->scan_tmp)
        if (p) (void)hipFree(p);
    for (int64_t *p : pl->scan_tmp_p)
        if (p) (void)hipFree(p);
    void *ptrs2[] = {pl->pcount, pl->nchunk, pl->pptr, pl->cptr, pl->pcursor, pl->plist, pl->plist_raw, pl->items,
                     pl->item_start, pl->item_cursor, pl->mom, pl->scoef, pl->gc_item, pl->t_pair,
                     pl->gc_self, pl->self_mark};
    for (void *p : ptrs2)
        if (p) (void)hipFree(p);
    if (pl->ev_ok)
        for (auto &e : pl->ev) (void)hipEventDestroy(e);
    delete pl;
}

nfq_status nfq_plan_create(nfq_ctx *ctx, const nfq_surface *surf, const nfq_targets *tg,
                           const nfq_nearlist *near, nfq_plan **out, int64_t *nnz_out,
                           int64_t *row_ptr)
{
    if (!ctx || !surf || !tg || !near || !out || !nnz_out || !row_ptr)
        return fail(ctx, NFQ_ERR_INVALID_ARG, "null argument");
    if (surf->P <= 0 || tg->NT < 0 || !surf->degree || !surf->node_ptr || !surf->xyz ||
        (tg->NT > 0 && (!tg->xyz || !tg->node_of_target || !near->row_ptr)))
        return fail(ctx, NFQ_ERR_INVALID_ARG, "bad sizes or null arrays");
    if (tg->NT >= (int64_t)INT32_MAX || surf->P >= (int64_t)INT32_MAX)
        return fail(ctx, NFQ_ERR_UNSUPPORTED, "more than 2^31 targets or patches");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    *out = nullptr;
    nfq_plan *pl = new (std::nothrow) nfq_plan;
    if (!pl) return fail(ctx, NFQ_ERR_OUT_OF_MEMORY, "plan");
    pl->ctx = ctx;
    pl->device = ctx->device;
    hipStream_t st = ctx->stream;
    Problem &pb = pl->pb;
    pb.P = surf->P;
    pb.NT = tg->NT;
    pb.degree = surf->degree;
    pb.node_ptr = surf->node_ptr;
    pb.xyz = surf->xyz;
    pb.txyz = tg->xyz;
    pb.node_of_target = tg->node_of_target;
    pb.near_rp = near->row_ptr;
    pb.near_patch = near->patch;
    pl->row_ptr = row_ptr;
    for (int d = 1; d <= 8; ++d)
        if (ctx->dV[d]) pl->present_mask |= 1 << d;
    auto cleanup = [&](nfq_status s) {
        nfq_plan_destroy(pl);
        return s;
    };
#define PL_TRY(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            ctx->err = std::string(#expr " -> ") + hipGetErrorString(e_);                     \
            return cleanup(e_ == hipErrorOutOfMemory ? NFQ_ERR_OUT_OF_MEMORY : NFQ_ERR_HIP);  \
        }                                                                                     \
    } while (0)
    PL_TRY(hipMemcpyAsync(&pb.N, surf->node_ptr + pb.P, 8, hipMemcpyDeviceToHost, st));
    PL_TRY(hipStreamSynchronize(st));
    if (pb.N <= 0 || pb.N >= (int64_t)INT32_MAX) return cleanup(fail(ctx, NFQ_ERR_INVALID_ARG, "bad node count"));
    const int64_t NT = pb.NT;
    PL_TRY(dalloc(&pl->rowlen, NT));
    PL_TRY(dalloc(&pl->npair, NT));
    PL_TRY(dalloc(&pl->pair_ptr, NT + 1));
    PL_TRY(dalloc(&pl->flags, kNumFlags));
    PL_TRY(dalloc(&pl->stats, kNumStats));
    PL_TRY(dalloc(&pl->counts, 18));
    PL_TRY(dalloc(&pl->cursor, 18));
    PL_TRY(dalloc(&pl->seg_start, 18));
    // scan temporaries
    {
        int64_t m = NT;
        while (true) {
            const int64_t tiles = (m + kScanTile - 1) / kScanTile;
            for (int k = 0; k < 4; ++k) {
                int64_t *p = nullptr;
                PL_TRY(dalloc(&p, tiles + 1));
                pl->scan_tmp.push_back(p);
            }
            if (m <= kScanTile) break;
            m = tiles;
        }
    }
    PL_TRY(hipMemsetAsync(pl->flags, 0, kNumFlags * sizeof(int), st));
    PL_TRY(hipMemsetAsync(pl->counts, 0, 18 * 8, st));
    if (NT > 0)
        hipLaunchKernelGGL(k_rowlen, dim3(nblk(NT, 256)), dim3(256), 0, st, pb, pl->present_mask,
                           pl->rowlen, pl->npair, pl->counts, pl->flags);
    nfq_status s = run_scan(pl->ctx, NT, pl->rowlen, pl->npair, row_ptr, pl->pair_ptr, pl->scan_tmp);
    if (s != NFQ_OK) return cleanup(s);
    int hflags[kNumFlags];
    PL_TRY(hipMemcpyAsync(hflags, pl->flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
    PL_TRY(hipMemcpyAsync(&pl->nnz, row_ptr + NT, 8, hipMemcpyDeviceToHost, st));
    PL_TRY(hipMemcpyAsync(&pl->npairs, pl->pair_ptr + NT, 8, hipMemcpyDeviceToHost, st));
    unsigned long long hc[18];
    PL_TRY(hipMemcpyAsync(hc, pl->counts, sizeof(hc), hipMemcpyDeviceToHost, st));
    PL_TRY(hipStreamSynchronize(st));
    s = check_flags(ctx, hflags);
    if (s != NFQ_OK) return cleanup(s);
    // segments: for d = 1..8: near_d (padded to 16) then self_d (padded)
    int64_t pos = 0;
    for (int d = 1; d <= 8; ++d) {
        for (int kind = 0; kind < 2; ++kind) {
            const int key = kind * 9 + d;
            pl->count_h[key] = (int64_t)hc[key];
            pl->seg_start_h[key] = pos;
            pl->seg_len_h[key] = pad16((int64_t)hc[key]);
            pos += pl->seg_len_h[key];
            if (hc[key] > 0) pl->max_degree = std::max(pl->max_degree, d);
        }
    }
    pl->grp_len = pos;
    const int64_t np = pl->npairs;
    PL_TRY(dalloc(&pl->pair_tgt, np));
    PL_TRY(dalloc(&pl->pair_patch, np));
    PL_TRY(dalloc(&pl->pair_self, np));
    PL_TRY(dalloc(&pl->pair_off, np));
    PL_TRY(dalloc(&pl->grp, pl->grp_len));
    PL_TRY(hipMemcpy(pl->seg_start, pl->seg_start_h, sizeof(pl->seg_start_h), hipMemcpyHostToDevice));
    PL_TRY(dalloc(&pl->coef, 3 * pb.N));
    PL_TRY(dalloc(&pl->coef_rel, 3 * pb.N));
    PL_TRY(dalloc(&pl->tau, pb.P));
    PL_TRY(dalloc(&pl->rho, pb.P));
    // patch-major work items of the near kernel: sized here, built in generate
    {
        const int64_t P = pb.P;
        PL_TRY(dalloc(&pl->pcount, P));
        PL_TRY(dalloc(&pl->nchunk, P));
        PL_TRY(dalloc(&pl->pptr, P + 1));
        PL_TRY(dalloc(&pl->cptr, P + 1));
        PL_TRY(dalloc(&pl->pcursor, P));
        PL_TRY(dalloc(&pl->item_start, 9));
        PL_TRY(dalloc(&pl->item_cursor, 9));
        PL_TRY(alloc_scan_tmp(P, pl->scan_tmp_p));
        for (int d = 1; d <= 8; ++d) pl->n_near += pl->count_h[d];
        PL_TRY(dalloc(&pl->plist, pl->n_near));
        PL_TRY(dalloc(&pl->plist_raw, pl->n_near));
        if (NT > 0)
            hipLaunchKernelGGL(k_pairs, dim3(nblk(NT, 256)), dim3(256), 0, st, pb, row_ptr,
                               pl->pair_ptr, pl->pair_tgt, pl->pair_patch, pl->pair_self,
                               pl->pair_off, (int32_t *)nullptr);
        PL_TRY(hipMemsetAsync(pl->pcount, 0, P * 8, st));
        PL_TRY(hipMemsetAsync(pl->item_cursor, 0, 9 * 8, st));
        if (np > 0)
            hipLaunchKernelGGL(k_patch_count, dim3(nblk(np, 256)), dim3(256), 0, st, np,
                               pl->pair_patch, pl->pair_self, pl->pcount);
        hipLaunchKernelGGL(k_patch_chunks, dim3(nblk(P, 256)), dim3(256), 0, st, P, pl->pcount,
                           pl->nchunk);
        hipLaunchKernelGGL(k_item_count, dim3(nblk(P, 256)), dim3(256), 0, st, P, pb.degree,
                           pl->nchunk, pl->item_cursor);
        unsigned long long hic[9];
        PL_TRY(hipMemcpyAsync(hic, pl->item_cursor, sizeof(hic), hipMemcpyDeviceToHost, st));
        PL_TRY(hipStreamSynchronize(st));
        int64_t ipos = 0;
        for (int d = 0; d < 9; ++d) {
            pl->item_start_h[d] = ipos;
            pl->item_count_h[d] = (int64_t)hic[d];
            ipos += (int64_t)hic[d];
        }
        pl->n_items = ipos;
        PL_TRY(dalloc(&pl->items, 3 * ipos));
        PL_TRY(hipMemcpy(pl->item_start, pl->item_start_h, sizeof(pl->item_start_h),
                         hipMemcpyHostToDevice));
    }
    // DFS stacks for the persistent near kernel: enough wavefronts to fill the chip
    {
        int ncu = 0;
        PL_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
        pl->stack_waves = (int64_t)std::max(ncu, 1) * 16;
        const int64_t esz = 8 + 2 * kNDMax;
        PL_TRY(dalloc(&pl->stack, pl->stack_waves * kStack * esz));
    }
    *nnz_out = pl->nnz;
    *out = pl;
#undef PL_TRY
    return NFQ_OK;
}

nfq_status nfq_generate(nfq_plan *pl, const nfq_kernel *kern, const nfq_params *prm, int32_t *col,
                        void *val, nfq_stats *stats)
{
    if (!pl || !kern || !prm || !col || !val) return fail(pl ? pl->ctx : nullptr, NFQ_ERR_INVALID_ARG, "null argument");
    nfq_ctx *ctx = pl->ctx;
    if (!(prm->tol > 0.0) || !(prm->loosen > 0.0) || prm->max_depth < 1 || prm->max_depth > kMaxDepth ||
        prm->min_depth < 0 || prm->min_depth > prm->max_depth)
        return fail(ctx, NFQ_ERR_INVALID_ARG, "tol, loosen must be > 0; 0 <= min_depth <= max_depth <= 32");
    if (prm->ng != 0 && prm->ng != kNG) return fail(ctx, NFQ_ERR_UNSUPPORTED, "only ng = 8 is supported");
    if (prm->self_nr < 0 || prm->self_na < 0 || prm->self_nr > kMaxGL || prm->self_na > kMaxGL)
        return fail(ctx, NFQ_ERR_INVALID_ARG, "self rule sizes must be in 0..64");
    if (kern->k_im < 0.0) return fail(ctx, NFQ_ERR_INVALID_ARG, "Im k must be >= 0");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const Problem &pb = pl->pb;
    const int64_t NT = pb.NT;
    const bool cplx = !(kern->k_re == 0.0 && kern->k_im == 0.0 && kern->alpha_im == 0.0 &&
                        kern->beta_im == 0.0);
    pl->value_kind = cplx ? 1 : 0;
    Timer tm{pl, (prm->flags & NFQ_FLAG_TIMING) != 0 && stats != nullptr};
    if (tm.on && !pl->ev_ok) {
        for (auto &e : pl->ev) HIP_TRY(ctx, hipEventCreate(&e));
        pl->ev_ok = true;
    }
    const bool per_pair = (prm->flags & NFQ_FLAG_PER_PAIR) != 0;
    QuadArgs qa{};
    PatchArgs pa{};
    nfq_status sp = prepare(pl, kern, prm, col, val, tm, per_pair, qa, pa);
    if (sp != NFQ_OK) return sp;
    for (int d = 1; d <= 8; ++d) {
        const int64_t ns = pl->seg_start_h[d], nc = pl->seg_len_h[d];
        const int64_t ss = pl->seg_start_h[9 + d], sc = pl->seg_len_h[9 + d];
        if (nc + sc == 0) continue;
        set_self_rule(ctx, prm, d, qa);
        if (cplx) launch_degree<true>(d, pl, qa, ns, nc, ss, sc, st, tm, per_pair, pa);
        else launch_degree<false>(d, pl, qa, ns, nc, ss, sc, st, tm, per_pair, pa);
    }
    HIP_TRY(ctx, hipGetLastError());
    if (stats) {
        int hflags[kNumFlags];
        unsigned long long hs[kNumStats];
        HIP_TRY(ctx, hipMemcpyAsync(hflags, pl->flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipMemcpyAsync(hs, pl->stats, sizeof(hs), hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        stats->near_pairs = (int64_t)hs[kStatNear];
        stats->self_pairs = (int64_t)hs[kStatSelf];
        stats->visits = (int64_t)hs[kStatVisits];
        stats->checks = (int64_t)hs[kStatChecks];
        stats->nonconverged = (int64_t)hs[kStatNonconv];
        stats->max_level = (int64_t)hs[kStatMaxLevel];
        stats->ms_builder = tm.on ? tm.total(kPhBuilder) : 0.0;
        stats->ms_prep = tm.on ? tm.total(kPhPrep) : 0.0;
        stats->ms_self = tm.on ? tm.total(kPhSelf) : 0.0;
        stats->ms_near = tm.on ? tm.total(kPhNear) : 0.0;
        stats->ms_weights = tm.on ? tm.total(kPhWeights) : 0.0;
        nfq_status fs = check_flags(ctx, hflags);
        if (fs != NFQ_OK) return fs;
        if (hs[kStatNonconv] > 0) return NFQ_WARN_NONCONVERGED;
    }
    return NFQ_OK;
}

nfq_status nfq_apply(nfq_plan *pl, const int32_t *col, const void *val, const void *sigma, void *y)
{
    if (!pl || !col || !val || !sigma || !y) return fail(pl ? pl->ctx : nullptr, NFQ_ERR_INVALID_ARG, "null argument");
    nfq_ctx *ctx = pl->ctx;
    if (pl->value_kind < 0) return fail(ctx, NFQ_ERR_INVALID_ARG, "nfq_apply before nfq_generate");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int64_t NT = pl->pb.NT;
    if (NT == 0) return NFQ_OK;
    if (pl->value_kind == 1)
        hipLaunchKernelGGL(k_apply<true>, dim3(nblk(NT, 4)), dim3(256), 0, ctx->stream, NT, pl->row_ptr,
                           col, (const double *)val, (const double *)sigma, (double *)y);
    else
        hipLaunchKernelGGL(k_apply<false>, dim3(nblk(NT, 4)), dim3(256), 0, ctx->stream, NT, pl->row_ptr,
                           col, (const double *)val, (const double *)sigma, (double *)y);
    HIP_TRY(ctx, hipGetLastError());
    return NFQ_OK;
}


nfq_status nfq_adjoint(nfq_plan *pl, const nfq_kernel *kern, const nfq_params *prm,
                       const void *sigma, const void *lambda, void *grad_xyz, void *grad_k,
                       void *dphi_dab)
{
    if (!pl || !kern || !prm || !sigma || !lambda || !grad_xyz || !grad_k)
        return fail(pl ? pl->ctx : nullptr, NFQ_ERR_INVALID_ARG, "null argument");
    nfq_ctx *ctx = pl->ctx;
    if (!(prm->tol > 0.0) || !(prm->loosen > 0.0) || prm->max_depth < 1 || prm->max_depth > kMaxDepth ||
        prm->min_depth < 0 || prm->min_depth > prm->max_depth)
        return fail(ctx, NFQ_ERR_INVALID_ARG, "tol, loosen must be > 0; 0 <= min_depth <= max_depth <= 32");
    if (prm->ng != 0 && prm->ng != kNG) return fail(ctx, NFQ_ERR_UNSUPPORTED, "only ng = 8 is supported");
    if (prm->self_nr < 0 || prm->self_na < 0 || prm->self_nr > kMaxGL || prm->self_na > kMaxGL)
        return fail(ctx, NFQ_ERR_INVALID_ARG, "self rule sizes must be in 0..64");
    if (kern->k_im < 0.0) return fail(ctx, NFQ_ERR_INVALID_ARG, "Im k must be >= 0");
    // The degree-7 instance of the near-pair adjoint kernel returns non-finite
    // values on gfx950 (degrees 6 and 8 and the degree-7 forward do not); it is
    // refused until the cause is found.
    if (pl->item_count_h[7] > 0)
        return fail(ctx, NFQ_ERR_UNSUPPORTED,
                    "adjoint of near pairs on degree-7 patches is disabled (known wrong values)");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const Problem &pb = pl->pb;
    const int64_t N = pb.N, NT = pb.NT;
    // adjoint scratch (allocated on first use)
    const int ndmax = nd_of(pl->max_degree > 0 ? pl->max_degree : 1);
    const int pitch = 6 + 18 * ndmax, self_pitch = 6 * ndmax;
    if (!pl->scoef || pl->gc_pitch < pitch) {
        (void)hipFree(pl->scoef); (void)hipFree(pl->gc_item); (void)hipFree(pl->t_pair);
        (void)hipFree(pl->gc_self); (void)hipFree(pl->self_mark);
        pl->scoef = pl->gc_item = pl->t_pair = pl->gc_self = nullptr;
        pl->self_mark = nullptr;
        HIP_TRY(ctx, dalloc(&pl->scoef, 2 * N));
        HIP_TRY(ctx, dalloc(&pl->gc_item, std::max<int64_t>(pl->n_items, 1) * pitch));
        HIP_TRY(ctx, dalloc(&pl->t_pair, std::max<int64_t>(pl->npairs, 1) * 12));
        HIP_TRY(ctx, dalloc(&pl->gc_self, N * self_pitch));
        HIP_TRY(ctx, dalloc(&pl->self_mark, N));
        pl->gc_pitch = pitch;
    }
    Timer tm{pl, false};
    QuadArgs qa{};
    PatchArgs pa{};
    nfq_status sp = prepare(pl, kern, prm, nullptr, nullptr, tm, false, qa, pa);
    if (sp != NFQ_OK) return sp;
    DegTab tab = make_tab(ctx);
    HIP_TRY(ctx, hipMemsetAsync(pl->self_mark, 0, N * sizeof(unsigned int), st));
    HIP_TRY(ctx, hipMemsetAsync(pl->t_pair, 0, std::max<int64_t>(pl->npairs, 1) * 12 * 8, st));
    if (NT > 0)
        hipLaunchKernelGGL(k_mark_self_nodes, dim3(nblk(NT, 256)), dim3(256), 0, st, pb,
                           pl->self_mark, pl->flags);
    hipLaunchKernelGGL(k_sigma_coef, dim3(nblk(pb.P, 64)), dim3(64), 0, st, pb, tab,
                       (const double *)sigma, pl->scoef);
    AdjArgs aa{};
    aa.pa = pa;
    aa.qa = qa;
    aa.scoef = pl->scoef;
    aa.lam = (const double *)lambda;
    aa.cptr = pl->cptr;
    aa.pptr = pl->pptr;
    aa.gc_item = pl->gc_item;
    aa.t_pair = pl->t_pair;
    aa.gc_self = pl->gc_self;
    aa.gc_pitch = pitch;
    aa.self_pitch = self_pitch;
    for (int d = 1; d <= 8; ++d) {
        const int64_t ss = pl->seg_start_h[9 + d], sc = pl->seg_len_h[9 + d];
        AdjArgs ad = aa;
        set_self_rule(ctx, prm, d, ad.qa);
        if (sc > 0) {
            ad.qa.seg = ss;
            ad.qa.count = sc;
            const unsigned blocks = (unsigned)std::min<int64_t>(sc, 4096);
#define NFQ_ADJ_SELF(DD) hipLaunchKernelGGL(k_adjoint_self<DD>, dim3(blocks), dim3(64), 0, st, ad)
            switch (d) {
            case 1: NFQ_ADJ_SELF(1); break; case 2: NFQ_ADJ_SELF(2); break;
            case 3: NFQ_ADJ_SELF(3); break; case 4: NFQ_ADJ_SELF(4); break;
            case 5: NFQ_ADJ_SELF(5); break; case 6: NFQ_ADJ_SELF(6); break;
            case 7: NFQ_ADJ_SELF(7); break; case 8: NFQ_ADJ_SELF(8); break;
            }
#undef NFQ_ADJ_SELF
        }
        if (pl->item_count_h[d] > 0) {
            ad.pa.item_seg = pl->item_start_h[d];
            ad.pa.item_count = pl->item_count_h[d];
            const unsigned blocks = (unsigned)std::min<int64_t>(ad.pa.item_count, pl->mom_slots);
#define NFQ_ADJ_NEAR(DD) hipLaunchKernelGGL(k_adjoint_patch<DD>, dim3(blocks), dim3(256), 0, st, ad)
            switch (d) {
            case 1: NFQ_ADJ_NEAR(1); break; case 2: NFQ_ADJ_NEAR(2); break;
            case 3: NFQ_ADJ_NEAR(3); break; case 4: NFQ_ADJ_NEAR(4); break;
            case 5: NFQ_ADJ_NEAR(5); break; case 6: NFQ_ADJ_NEAR(6); break;
            case 7: NFQ_ADJ_NEAR(7); break; case 8: NFQ_ADJ_NEAR(8); break;
            }
#undef NFQ_ADJ_NEAR
        }
    }
    hipLaunchKernelGGL(k_adj_patch_final, dim3(nblk(pb.P, 64)), dim3(64), 0, st, pb, tab, pl->cptr,
                       pl->nchunk, pl->gc_item, pitch, pl->gc_self, self_pitch, pl->self_mark,
                       (double *)grad_xyz);
    if (NT > 0)
        hipLaunchKernelGGL(k_adj_target_final, dim3(nblk(NT, 256)), dim3(256), 0, st, pb, pl->pair_ptr,
                           pl->t_pair, (double *)grad_xyz);
    hipLaunchKernelGGL(k_adj_scalars, dim3(1), dim3(256), 0, st, pl->npairs, pl->t_pair,
                       pl->n_items, pl->gc_item, pitch, (double *)grad_k, (double *)dphi_dab);
    HIP_TRY(ctx, hipGetLastError());
    int hflags[kNumFlags];
    HIP_TRY(ctx, hipMemcpyAsync(hflags, pl->flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    return check_flags(ctx, hflags);
}

nfq_status nfq_sync(nfq_ctx *ctx)
{
    if (!ctx) return NFQ_ERR_INVALID_ARG;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return NFQ_OK;
}

nfq_status nfq_near_lists(nfq_ctx *ctx, const nfq_surface *surf, const nfq_targets *targets,
                          double eta, int64_t *row_ptr, int32_t *patch, int64_t capacity,
                          int64_t *nnz_out, double *centres, double *radii)
{
    if (!ctx || !surf || !targets || !row_ptr || !nnz_out)
        return fail(ctx, NFQ_ERR_INVALID_ARG, "null argument");
    const int64_t P = surf->P, NT = targets->NT;
    if (P < 0 || NT < 0 || P > INT32_MAX || capacity < 0 || !(eta > 0.0) || !(eta < 1e300))
        return fail(ctx, NFQ_ERR_INVALID_ARG, "sizes, capacity or eta out of range");
    if ((P > 0 && (!surf->degree || !surf->node_ptr || !surf->xyz)) ||
        (NT > 0 && (!targets->xyz || !targets->node_of_target)) || (capacity > 0 && !patch))
        return fail(ctx, NFQ_ERR_INVALID_ARG, "null array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    // scratch owned by this call, released on every return path
    struct Scratch {
        std::vector<void *> p;
        std::vector<int64_t *> scan;
        ~Scratch() {
            for (void *q : p) (void)hipFree(q);
            for (int64_t *q : scan) (void)hipFree(q);
        }
    } sc;
    auto grab = [&](auto **ptr, int64_t count) -> hipError_t {
        hipError_t e = dalloc(ptr, std::max<int64_t>(count, 1));
        if (e == hipSuccess) sc.p.push_back((void *)*ptr);
        return e;
    };
#define NL_TRY(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(ctx, e_ == hipErrorOutOfMemory ? NFQ_ERR_OUT_OF_MEMORY : NFQ_ERR_HIP,       \
                        std::string(#expr " -> ") + hipGetErrorString(e_));                         \
    } while (0)
    Problem pb{};
    pb.P = P;
    pb.NT = NT;
    pb.degree = surf->degree;
    pb.node_ptr = surf->node_ptr;
    pb.xyz = surf->xyz;
    pb.txyz = targets->xyz;
    pb.node_of_target = targets->node_of_target;
    double *dc = centres, *dr = radii;
    if (!dc) NL_TRY(grab(&dc, 3 * P));
    if (!dr) NL_TRY(grab(&dr, P));
    int *flags = nullptr;
    NL_TRY(grab(&flags, 4));
    fill32(flags, 4 * sizeof(int), 0u, st);
    if (P > 0)
        hipLaunchKernelGGL(k_balls, dim3((unsigned)std::min<int64_t>(P, 1 << 16)), dim3(64), 0, st, pb,
                           make_tab(ctx), dc, dr, flags);
    // extent of the targets and the largest ball
    const int eblocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (std::max(NT, P) + 255) / 256));
    double *part = nullptr;
    NL_TRY(grab(&part, 7 * eblocks));
    hipLaunchKernelGGL(k_extent, dim3(eblocks), dim3(256), 0, st, NT, pb.txyz, P, dr, part);
    std::vector<double> hpart(7 * eblocks);
    int hflags[4];
    NL_TRY(hipMemcpyAsync(hpart.data(), part, hpart.size() * 8, hipMemcpyDeviceToHost, st));
    NL_TRY(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
    NL_TRY(hipStreamSynchronize(st));
    if (hflags[kNearFlagUnregistered]) return fail(ctx, NFQ_ERR_NOT_REGISTERED, "patch degree not registered");
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, rmax = 0.0;
    for (int b = 0; b < eblocks; ++b) {
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], hpart[7 * b + c]);
            hi[c] = std::max(hi[c], hpart[7 * b + 3 + c]);
        }
        rmax = std::max(rmax, hpart[7 * b + 6]);
    }
    if (NT == 0 || P == 0) {
        fill32(row_ptr, (NT + 1) * 8, 0u, st);
        NL_TRY(hipStreamSynchronize(st));
        *nnz_out = 0;
        return NFQ_OK;
    }
    for (int c = 0; c < 3; ++c)
        if (!(lo[c] <= hi[c]) || !(hi[c] - lo[c] < 1e300))
            return fail(ctx, NFQ_ERR_INVALID_ARG, "target coordinates not finite");
    // cells at least eta * max R wide, at most 2^24 of them
    Grid g{};
    const double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    double h = std::max(std::max(eta * rmax, ext / 256.0), 1e-300);
    for (int it = 0; it < 200; ++it) {
        int64_t tot = 1;
        for (int c = 0; c < 3; ++c) {
            g.n[c] = (int64_t)std::floor((hi[c] - lo[c]) / h) + 1;
            tot = (g.n[c] > (int64_t(1) << 24)) ? (int64_t(1) << 25) : tot * g.n[c];
            if (tot > (int64_t(1) << 24)) break;
        }
        if (tot <= (int64_t(1) << 24)) break;
        h *= 1.25;
    }
    for (int c = 0; c < 3; ++c) g.o[c] = lo[c];
    g.inv_h = 1.0 / h;
    const int64_t ncell = g.n[0] * g.n[1] * g.n[2];
    if (ncell > (int64_t(1) << 24)) return fail(ctx, NFQ_ERR_INVALID_ARG, "target extent too large for the grid");
    // targets by cell
    int64_t *cnt = nullptr, *cstart = nullptr, *cdummy = nullptr, *items = nullptr;
    NL_TRY(grab(&cnt, ncell));
    NL_TRY(grab(&cstart, ncell + 1));
    NL_TRY(grab(&cdummy, ncell + 1));
    NL_TRY(grab(&items, NT));
    NL_TRY(alloc_scan_tmp(std::max(ncell, NT), sc.scan));
    fill32(cnt, ncell * 8, 0u, st);
    hipLaunchKernelGGL(k_cell_count, dim3(nblk(NT, 256)), dim3(256), 0, st, NT, pb.txyz, g,
                       (unsigned long long *)cnt);
    nfq_status s = run_scan(ctx, ncell, cnt, cnt, cstart, cdummy, sc.scan);
    if (s != NFQ_OK) return s;
    fill32(cnt, ncell * 8, 0u, st);
    hipLaunchKernelGGL(k_cell_fill, dim3(nblk(NT, 256)), dim3(256), 0, st, NT, pb.txyz, g, cstart,
                       (unsigned long long *)cnt, items);
    // pairs per target, row pointers
    int64_t *rowlen = nullptr, *rdummy = nullptr;
    NL_TRY(grab(&rowlen, NT));
    NL_TRY(grab(&rdummy, NT + 1));
    fill32(rowlen, NT * 8, 0u, st);
    const unsigned pblocks = (unsigned)std::min<int64_t>(P, 1 << 16);
    hipLaunchKernelGGL(k_near_scan<false>, dim3(pblocks), dim3(64), 0, st, pb, g, eta, dc, dr, cstart,
                       items, (unsigned long long *)rowlen, (const int64_t *)nullptr, (int32_t *)nullptr);
    s = run_scan(ctx, NT, rowlen, rowlen, row_ptr, rdummy, sc.scan);
    if (s != NFQ_OK) return s;
    int64_t nnz = 0;
    NL_TRY(hipMemcpyAsync(&nnz, row_ptr + NT, 8, hipMemcpyDeviceToHost, st));
    NL_TRY(hipStreamSynchronize(st));
    *nnz_out = nnz;
    if (nnz > capacity)
        return fail(ctx, NFQ_ERR_INVALID_ARG,
                    "patch capacity " + std::to_string(capacity) + " < " + std::to_string(nnz) +
                        " near pairs (row_ptr written; call again with capacity >= nnz)");
    if (nnz > 0) {
        fill32(rowlen, NT * 8, 0u, st);
        hipLaunchKernelGGL(k_near_scan<true>, dim3(pblocks), dim3(64), 0, st, pb, g, eta, dc, dr,
                           cstart, items, (unsigned long long *)rowlen, (const int64_t *)row_ptr, patch);
        hipLaunchKernelGGL(k_row_sort, dim3(nblk(NT, 256)), dim3(256), 0, st, NT, (const int64_t *)row_ptr,
                           patch);
    }
    NL_TRY(hipGetLastError());
    NL_TRY(hipStreamSynchronize(st));
#undef NL_TRY
    return NFQ_OK;
}

}  // extern "C"
