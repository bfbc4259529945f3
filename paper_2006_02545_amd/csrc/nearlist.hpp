// nearlist.hpp -- near lists T_eta(x_t) on the device (near-field definitions
// of Section 4; lists by target as in Section 5.2).
//
// Patch j's ball: centre c_j = parametric mean of its chart, (1/|T0|) int_T0
// X du dv = sqrt(2) x_00 (the constant Koornwinder function K_00 = sqrt(2) is
// the only one with a nonzero integral), radius R_j = max |X(u,v) - c_j| over
// the lattice (i/64, k/64), i + k <= 64, of T0.  Target t is near patch j when
// |x_t - c_j| < eta R_j and j is not the target's own patch.
//
// Targets are binned into a uniform grid whose cells are at least eta max R
// wide (counting sort by cell); one wavefront per patch scans the cells that
// its ball's bounding box touches, once to count the pairs of every target
// and once to scatter the patch ids into the rows, which are then sorted.
#pragma once

#include "kernels.hpp"

namespace nfq {

constexpr int kBallLattice = 64;
constexpr int kNearFlagUnregistered = 0;

// Ball of patch j (one wavefront; s_cf holds 3 * 45 doubles).
template <int D>
__device__ void patch_ball(const Problem &pb, const DegTab &tab, int64_t j, double *s_cf, int lane,
                           double *centres, double *radii)
{
    constexpr int ND = nd_of(D);
    const double *V = tab.V[D];
    const double *x = pb.xyz + 3 * pb.node_ptr[j];
    for (int a = lane; a < ND; a += 64) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int l = 0; l < ND; ++l) {
            const double v = V[a * ND + l];
            s0 = __builtin_fma(v, x[3 * l + 0], s0);
            s1 = __builtin_fma(v, x[3 * l + 1], s1);
            s2 = __builtin_fma(v, x[3 * l + 2], s2);
        }
        s_cf[a] = s0;
        s_cf[ND + a] = s1;
        s_cf[2 * ND + a] = s2;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double sq2 = 1.4142135623730951;
    const double c0 = sq2 * s_cf[0], c1 = sq2 * s_cf[ND], c2 = sq2 * s_cf[2 * ND];
    constexpr int NL = kBallLattice + 1;
    double r2max = 0.0;
    for (int idx = lane; idx < NL * NL; idx += 64) {
        const int i = idx / NL, k = idx - i * NL;
        if (i + k > kBallLattice) continue;
        const double u = i * (1.0 / kBallLattice), v = k * (1.0 / kBallLattice);
        double X0 = 0.0, X1 = 0.0, X2 = 0.0;
        koorn_visit<D>(u, v, [&](int a, double kv, double, double) {
            X0 = __builtin_fma(s_cf[a], kv, X0);
            X1 = __builtin_fma(s_cf[ND + a], kv, X1);
            X2 = __builtin_fma(s_cf[2 * ND + a], kv, X2);
        });
        const double d0 = X0 - c0, d1 = X1 - c1, d2 = X2 - c2;
        r2max = __builtin_fmax(r2max, d0 * d0 + d1 * d1 + d2 * d2);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) r2max = __builtin_fmax(r2max, __shfl_xor(r2max, off, 64));
    if (lane == 0) {
        centres[3 * j] = c0;
        centres[3 * j + 1] = c1;
        centres[3 * j + 2] = c2;
        radii[j] = __builtin_sqrt(r2max);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64) void k_balls(Problem pb, DegTab tab, double *centres, double *radii,
                                              int *flags)
{
    __shared__ double s_cf[3 * 45];
    const int lane = threadIdx.x;
    for (int64_t j = blockIdx.x; j < pb.P; j += gridDim.x) {
        const int d = pb.degree[j];
        if (d < 1 || d > 8 || !tab.present[d]) {
            if (lane == 0) flags[kNearFlagUnregistered] = 1;
            continue;
        }
        switch (d) {
        case 1: patch_ball<1>(pb, tab, j, s_cf, lane, centres, radii); break;
        case 2: patch_ball<2>(pb, tab, j, s_cf, lane, centres, radii); break;
        case 3: patch_ball<3>(pb, tab, j, s_cf, lane, centres, radii); break;
        case 4: patch_ball<4>(pb, tab, j, s_cf, lane, centres, radii); break;
        case 5: patch_ball<5>(pb, tab, j, s_cf, lane, centres, radii); break;
        case 6: patch_ball<6>(pb, tab, j, s_cf, lane, centres, radii); break;
        case 7: patch_ball<7>(pb, tab, j, s_cf, lane, centres, radii); break;
        default: patch_ball<8>(pb, tab, j, s_cf, lane, centres, radii); break;
        }
    }
}

// Per-block partial extents: min and max of the target coordinates and the
// largest ball radius; part[block][7] = (min xyz, max xyz, max R).
__global__ __launch_bounds__(256) void k_extent(int64_t NT, const double *txyz, int64_t P,
                                                const double *radii, double *part)
{
    __shared__ double s[7][256];
    double v[7] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < NT; t += stride)
        for (int c = 0; c < 3; ++c) {
            const double x = txyz[3 * t + c];
            v[c] = __builtin_fmin(v[c], x);
            v[3 + c] = __builtin_fmax(v[3 + c], x);
        }
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P; j += stride)
        v[6] = __builtin_fmax(v[6], radii[j]);
    for (int c = 0; c < 7; ++c) s[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int c = 0; c < 7; ++c) {
                const double o = s[c][threadIdx.x + h];
                s[c][threadIdx.x] = (c < 3) ? __builtin_fmin(s[c][threadIdx.x], o)
                                            : __builtin_fmax(s[c][threadIdx.x], o);
            }
        __syncthreads();
    }
    if (threadIdx.x < 7) part[7 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

struct Grid {
    double o[3];
    double inv_h;
    int64_t n[3];
};

__device__ __forceinline__ int64_t grid_coord(double x, double o, double inv_h, int64_t n)
{
    const double f = __builtin_floor((x - o) * inv_h);
    if (!(f > 0.0)) return 0;                       // also NaN
    return f >= (double)(n - 1) ? n - 1 : (int64_t)f;
}

__device__ __forceinline__ int64_t grid_cell(const Grid &g, const double *x)
{
    const int64_t i = grid_coord(x[0], g.o[0], g.inv_h, g.n[0]);
    const int64_t k = grid_coord(x[1], g.o[1], g.inv_h, g.n[1]);
    const int64_t m = grid_coord(x[2], g.o[2], g.inv_h, g.n[2]);
    return (m * g.n[1] + k) * g.n[0] + i;
}

__global__ __launch_bounds__(256) void k_cell_count(int64_t NT, const double *txyz, Grid g,
                                                    unsigned long long *cnt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NT) return;
    atomicAdd(&cnt[grid_cell(g, txyz + 3 * t)], 1ull);
}

__global__ __launch_bounds__(256) void k_cell_fill(int64_t NT, const double *txyz, Grid g,
                                                   const int64_t *start, unsigned long long *cursor,
                                                   int64_t *items)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NT) return;
    const int64_t c = grid_cell(g, txyz + 3 * t);
    items[start[c] + (int64_t)atomicAdd(&cursor[c], 1ull)] = t;
}

// One wavefront per patch: every target in the cells of the ball's bounding
// box is tested.  FILL = false counts pairs per target into `cnt`; FILL = true
// writes patch ids at row_ptr[t] + (per-target cursor in `cnt`).
template <bool FILL>
__global__ __launch_bounds__(64) void k_near_scan(Problem pb, Grid g, double eta,
                                                  const double *centres, const double *radii,
                                                  const int64_t *start, const int64_t *items,
                                                  unsigned long long *cnt, const int64_t *row_ptr,
                                                  int32_t *patch)
{
    const int lane = threadIdx.x;
    for (int64_t j = blockIdx.x; j < pb.P; j += gridDim.x) {
        const double c[3] = {centres[3 * j], centres[3 * j + 1], centres[3 * j + 2]};
        const double r = eta * radii[j];
        const int64_t n0 = pb.node_ptr[j], n1 = pb.node_ptr[j + 1];
        int64_t lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = grid_coord(c[a] - r, g.o[a], g.inv_h, g.n[a]);
            hi[a] = grid_coord(c[a] + r, g.o[a], g.inv_h, g.n[a]);
        }
        for (int64_t m = lo[2]; m <= hi[2]; ++m)
            for (int64_t k = lo[1]; k <= hi[1]; ++k)
                for (int64_t i = lo[0]; i <= hi[0]; ++i) {
                    const int64_t cell = (m * g.n[1] + k) * g.n[0] + i;
                    const int64_t e = start[cell + 1];
                    for (int64_t q = start[cell] + lane; q < e; q += 64) {
                        const int64_t t = items[q];
                        const double d0 = pb.txyz[3 * t] - c[0], d1 = pb.txyz[3 * t + 1] - c[1];
                        const double d2 = pb.txyz[3 * t + 2] - c[2];
                        const double dist = __builtin_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                        if (!(dist < r)) continue;
                        const int64_t nt = pb.node_of_target[t];
                        if (nt >= n0 && nt < n1) continue;   // the target's own patch
                        if (!FILL) {
                            atomicAdd(&cnt[t], 1ull);
                        } else {
                            const int64_t pos = row_ptr[t] + (int64_t)atomicAdd(&cnt[t], 1ull);
                            patch[pos] = (int32_t)j;
                        }
                    }
                }
    }
}

// Rows in ascending patch order (insertion sort; rows are short).
__global__ __launch_bounds__(256) void k_row_sort(int64_t NT, const int64_t *row_ptr, int32_t *patch)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NT) return;
    const int64_t b = row_ptr[t], e = row_ptr[t + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        const int32_t v = patch[i];
        int64_t k = i - 1;
        while (k >= b && patch[k] > v) {
            patch[k + 1] = patch[k];
            --k;
        }
        patch[k + 1] = v;
    }
}

}  // namespace nfq
