// k_direct.hip -- softened direct summation of g, j and T (all sources act
// on each listed target), in FP64 or with FP32 pair terms.
//
// Layout: a workgroup of 256 threads owns 256 targets (one per lane) and one
// contiguous chunk of sources; the chunk is streamed through LDS in tiles of
// 256 sources (coalesced loads, every lane then reads the tile as an LDS
// broadcast).  Small problems are split over sources (grid.y) so that the
// launch fills all 256 CUs; each split writes FP64 partial sums, which a
// second kernel adds in a fixed order (bit-reproducible results).
//
// FP32-pair mode: the separation d = x_j - x_i is formed in FP64 and rounded
// once to FP32 (the exact relative coordinate), the pair term is computed in
// FP32, and each tile's FP32 partial sum is folded into FP64 accumulators.
//
// Periodic cube of side L (kPer): d is replaced by its nearest image
// d - L rint(d / L), in FP64, before anything else.
//
// Per-particle softening (kSoft): each pair's f and D are the means of the
// target's and the source's kernels (hs, input order).
#include "ag_internal.h"
#include "pair.h"

namespace {

constexpr int kT = 256;          // targets per workgroup = sources per LDS tile
constexpr int kParts = 12;       // g (3), j (3), S (6)

__device__ __forceinline__ double near_img(double d, double L) { return d - L * rint(d / L); }

template <bool kFP64, bool kPer, bool kSoft>
__global__ void __launch_bounds__(kT) k_direct(int64_t n, const double* __restrict__ x,
                                               const double* __restrict__ v,
                                               const double* __restrict__ m,
                                               const double* __restrict__ hs,
                                               const int32_t* __restrict__ idx, int64_t n_act,
                                               double h, double L, int64_t chunk,
                                               double* __restrict__ part,
                                               int32_t* __restrict__ flags) {
    __shared__ double s_x[kT], s_y[kT], s_z[kT];
    __shared__ float s_vx[kT], s_vy[kT], s_vz[kT];
    __shared__ double s_dvx[kFP64 ? kT : 1], s_dvy[kFP64 ? kT : 1], s_dvz[kFP64 ? kT : 1];
    __shared__ double s_m[kT];
    __shared__ double s_h[kSoft ? kT : 1];

    const int64_t k = (int64_t)blockIdx.x * kT + threadIdx.x;
    const bool live = k < n_act;
    int64_t i = -1;
    if (live) {
        i = idx ? (int64_t)idx[k] : k;
        if (i < 0 || i >= n) {
            atomicOr(flags, AGF_BADINDEX);
            i = -1;
        }
    }
    double xi = 0, yi = 0, zi = 0, vxi = 0, vyi = 0, vzi = 0, hi_ = 1.0;
    if (i >= 0) {
        xi = x[3 * i]; yi = x[3 * i + 1]; zi = x[3 * i + 2];
        vxi = v[3 * i]; vyi = v[3 * i + 1]; vzi = v[3 * i + 2];
        if (kSoft) hi_ = hs[i];
    }
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;

    PairAcc<double> A;
    A.zero();
    const double h2 = h * h, hinv = 1.0 / h;
    const float h2f = (float)h2, hinvf = (float)hinv;
    const float vxf = (float)vxi, vyf = (float)vyi, vzf = (float)vzi;

    for (int64_t t0 = j0; t0 < j1; t0 += kT) {
        const int64_t js = t0 + threadIdx.x;
        __syncthreads();
        if (js < j1) {
            s_x[threadIdx.x] = x[3 * js];
            s_y[threadIdx.x] = x[3 * js + 1];
            s_z[threadIdx.x] = x[3 * js + 2];
            s_m[threadIdx.x] = m[js];
            if (kSoft) s_h[threadIdx.x] = hs[js];
            if (kFP64) {
                s_dvx[threadIdx.x] = v[3 * js];
                s_dvy[threadIdx.x] = v[3 * js + 1];
                s_dvz[threadIdx.x] = v[3 * js + 2];
            } else {
                s_vx[threadIdx.x] = (float)v[3 * js];
                s_vy[threadIdx.x] = (float)v[3 * js + 1];
                s_vz[threadIdx.x] = (float)v[3 * js + 2];
            }
        }
        __syncthreads();
        const int cnt = (int)((j1 - t0) < kT ? (j1 - t0) : kT);
        if (i < 0) continue;
        if (kFP64) {
            for (int q = 0; q < cnt; ++q) {
                const double mj = (t0 + q == i) ? 0.0 : s_m[q];   // self pair excluded
                double dx = s_x[q] - xi, dy = s_y[q] - yi, dz = s_z[q] - zi;
                if (kPer) {
                    dx = near_img(dx, L);
                    dy = near_img(dy, L);
                    dz = near_img(dz, L);
                }
                if (kSoft)
                    pair_interact_soft<double>(dx, dy, dz, s_dvx[q] - vxi, s_dvy[q] - vyi, s_dvz[q] - vzi, mj, hi_,
                                               s_h[q], A);
                else
                    pair_interact<double>(dx, dy, dz, s_dvx[q] - vxi, s_dvy[q] - vyi, s_dvz[q] - vzi, mj, h2,
                                          hinv, A);
            }
        } else {
            PairAcc<float> B;
            B.zero();
            for (int q = 0; q < cnt; ++q) {
                const float mj = (t0 + q == i) ? 0.0f : (float)s_m[q];
                double dx = s_x[q] - xi, dy = s_y[q] - yi, dz = s_z[q] - zi;
                if (kPer) {
                    dx = near_img(dx, L);
                    dy = near_img(dy, L);
                    dz = near_img(dz, L);
                }
                if (kSoft)
                    pair_interact_soft<float>((float)dx, (float)dy, (float)dz, s_vx[q] - vxf, s_vy[q] - vyf,
                                              s_vz[q] - vzf, mj, (float)hi_, (float)s_h[q], B);
                else
                    pair_interact<float>((float)dx, (float)dy, (float)dz, s_vx[q] - vxf, s_vy[q] - vyf,
                                         s_vz[q] - vzf, mj, h2f, hinvf, B);
            }
            A.ax += B.ax; A.ay += B.ay; A.az += B.az;
            A.jx += B.jx; A.jy += B.jy; A.jz += B.jz;
            A.sxx += B.sxx; A.syy += B.syy; A.szz += B.szz;
            A.sxy += B.sxy; A.sxz += B.sxz; A.syz += B.syz;
        }
    }
    if (!live) return;
    // partials in [split][component][target] order (coalesced stores)
    double* p = part + (int64_t)blockIdx.y * kParts * n_act + k;
    const double vals[kParts] = {A.ax, A.ay, A.az, A.jx, A.jy, A.jz,
                                 A.sxx, A.syy, A.szz, A.sxy, A.sxz, A.syz};
#pragma unroll
    for (int c = 0; c < kParts; ++c) p[(int64_t)c * n_act] = vals[c];
}

// fixed-order sum of the source splits, scaled by G, scattered to the rows
__global__ void k_direct_reduce(int64_t n, const int32_t* __restrict__ idx, int64_t n_act, int nsplit,
                                const double* __restrict__ part, double G, double* __restrict__ acc,
                                double* __restrict__ jerk, double* __restrict__ tidal) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_act;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = idx ? (int64_t)idx[k] : k;
        if (i < 0 || i >= n) continue;
        double s[kParts];
#pragma unroll
        for (int c = 0; c < kParts; ++c) s[c] = 0.0;
        for (int q = 0; q < nsplit; ++q) {
            const double* p = part + (int64_t)q * kParts * n_act + k;
#pragma unroll
            for (int c = 0; c < kParts; ++c) s[c] += p[(int64_t)c * n_act];
        }
        if (acc) {
            acc[3 * i] = G * s[0]; acc[3 * i + 1] = G * s[1]; acc[3 * i + 2] = G * s[2];
        }
        if (jerk) {
            jerk[3 * i] = G * s[3]; jerk[3 * i + 1] = G * s[4]; jerk[3 * i + 2] = G * s[5];
        }
        if (tidal) {
#pragma unroll
            for (int c = 0; c < 6; ++c) tidal[6 * i + c] = -G * s[6 + c];
        }
    }
}

}  // namespace

int ag_launch_direct(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                     const int32_t* idx, int64_t n_act, double eps, double G, int precision,
                     double* acc, double* jerk, double* tidal) {
    const int64_t tblocks = (n_act + kT - 1) / kT;
    const int64_t max_split = (n + kT - 1) / kT;
    int64_t nsplit = (2048 + tblocks - 1) / tblocks;   // aim at >= 2048 workgroups
    if (nsplit > max_split) nsplit = max_split;
    if (nsplit > 65535) nsplit = 65535;
    if (nsplit < 1) nsplit = 1;
    int64_t chunk = (n + nsplit - 1) / nsplit;
    chunk = (chunk + kT - 1) / kT * kT;
    nsplit = (n + chunk - 1) / chunk;
    AG_TRY(ag_ensure(c, c->direct_part, (size_t)nsplit * kParts * (size_t)n_act * sizeof(double)));
    double* part = c->direct_part.as<double>();
    PhaseScope phase(c, AG_PHASE_DIRECT);
    dim3 grid((unsigned)tblocks, (unsigned)nsplit);
    const double L = c->box;
    int32_t* fl = c->dflags.as<int32_t>();
    hipStream_t st = c->stream;
    const bool fp64 = precision == AG_FP64, per = L > 0.0, soft = c->soft_n > 0;
    const double* hs = soft ? c->soft_h.as<double>() : nullptr;
#define AG_DIRECT(A, B, C)                                                                                       \
    hipLaunchKernelGGL((k_direct<A, B, C>), grid, dim3(kT), 0, st, n, x, v, m, hs, idx, n_act, eps, L, chunk, part, \
                       fl)
    if (fp64) {
        if (per) { if (soft) AG_DIRECT(true, true, true); else AG_DIRECT(true, true, false); }
        else { if (soft) AG_DIRECT(true, false, true); else AG_DIRECT(true, false, false); }
    } else {
        if (per) { if (soft) AG_DIRECT(false, true, true); else AG_DIRECT(false, true, false); }
        else { if (soft) AG_DIRECT(false, false, true); else AG_DIRECT(false, false, false); }
    }
#undef AG_DIRECT
    int64_t rb = (n_act + 255) / 256;
    if (rb > 4096) rb = 4096;
    hipLaunchKernelGGL(k_direct_reduce, dim3((unsigned)rb), dim3(256), 0, c->stream, n, idx, n_act,
                       (int)nsplit, part, G, acc, jerk, tidal);
    // every listed target received a fresh force
    return AG_OK;
}
