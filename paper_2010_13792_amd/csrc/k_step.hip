// k_step.hip -- per-particle kernels of the adaptive scheme: the tidal
// timestep and its block bin (Eq. 7), the force-age counter and update test
// (Eq. 3, Eq. 4) with stream compaction, and the jerk predictor (Eq. 6);
// plus the device-wide exclusive scan used across the library.
//
// This file is compiled with -ffp-contract=off: the bin decision and the
// predictor are defined operation by operation (each rounded once), so the
// compiler must not fuse a multiply into an add.
//
// All kernels here are HBM-bound streaming passes: one thread per row,
// consecutive threads on consecutive rows (coalesced), grid-stride loops.
#include "ag_internal.h"

namespace {

constexpr int kThreads = 256;

int grid_for(int64_t n, int threads = kThreads) {
    int64_t b = (n + threads - 1) / threads;
    if (b > 8192) b = 8192;   // 32 blocks per CU over 256 CUs; loops cover the rest
    return (int)(b < 1 ? 1 : b);
}

// ---------------------------------------------------------------------------
// Eq. 7 tidal timestep and power-of-two bin
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tidal_bin(double n2, double eta, double dt_max, int k_max) {
    // Q = (dt_max / dt_grav)^4 = n2 dt_max^4 / (6 eta^2), one rounding per op
    double a = dt_max * dt_max;
    double b = a * a;
    double e2 = eta * eta;
    double den = 6.0 * e2;
    double num = n2 * b;
    double Q = num / den;
    if (!(Q == Q) || Q > 1.7976931348623157e308) return k_max;
    if (Q <= 0.0) return 0;
    int e;
    double fr = frexp(Q, &e);            // Q = fr 2^e, fr in [1/2, 1)
    int mexp = (fr == 0.5) ? e - 1 : e;  // least integer m with Q <= 2^m
    int k = mexp <= 0 ? 0 : (mexp + 3) / 4;
    return k > k_max ? k_max : k;
}

// rows idx[0 .. n_rows), or with n_dev set idx[0 .. *n_dev) (a count outside
// [0, n_rows] raises the flag and processes none)
__global__ void k_timestep(int64_t n_rows, const int64_t* __restrict__ n_dev, const int32_t* __restrict__ idx,
                           int64_t n, const double* __restrict__ tidal, double eta, double sqrt_eta,
                           double dt_max, int k_max, double* __restrict__ dt,
                           int8_t* __restrict__ bin, int32_t* __restrict__ flags) {
    if (n_dev) {
        const int64_t v = *n_dev;
        const bool bad = v < 0 || v > n_rows;
        if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, AGF_BADINDEX);
        n_rows = bad ? 0 : v;
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_rows;
         k += (int64_t)gridDim.x * blockDim.x) {
        int64_t r = idx ? (int64_t)idx[k] : k;
        if (r < 0 || r >= n) {
            atomicOr(flags, AGF_BADINDEX);
            continue;
        }
        const double* t = tidal + 6 * r;
        double t0 = t[0], t1 = t[1], t2 = t[2], t3 = t[3], t4 = t[4], t5 = t[5];
        double d2 = t0 * t0 + t1 * t1;
        d2 = d2 + t2 * t2;
        double o2 = t3 * t3 + t4 * t4;
        o2 = o2 + t5 * t5;
        double n2 = d2 + 2.0 * o2;
        dt[r] = (n2 > 0.0) ? sqrt_eta * pow(n2 / 6.0, -0.25) : __builtin_huge_val();
        bin[r] = (int8_t)tidal_bin(n2, eta, dt_max, k_max);
    }
}

// ---------------------------------------------------------------------------
// Eq. 3 / Eq. 4 bookkeeping: flag due particles, reset their counters
// ---------------------------------------------------------------------------
__global__ void k_select(int64_t n, int64_t* __restrict__ tf, const int8_t* __restrict__ bin,
                         int64_t step_ticks, int tick_bin, double q_f,
                         int32_t* __restrict__ flag) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int k = bin[i];
        k = k < 0 ? 0 : (k > tick_bin ? tick_bin : k);
        int64_t span = (int64_t)1 << (tick_bin - k);
        int64_t t = tf[i] + step_ticks;            // Eq. 3
        double thresh = q_f * (double)span;
        int due = ((double)t >= thresh) ? 1 : 0;   // Eq. 4, inclusive
        tf[i] = due ? 0 : t;
        flag[i] = due;
    }
}

__global__ void k_compact(int64_t n, const int32_t* __restrict__ flag,
                          const int32_t* __restrict__ off, int32_t* __restrict__ out,
                          int64_t* __restrict__ count, double* __restrict__ t0, double t) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (flag[i]) {
            out[off[i]] = (int32_t)i;
            if (t0) t0[i] = t;
        }
    }
    if (count && blockIdx.x == 0 && threadIdx.x == 0) *count = (int64_t)off[n];
}

// leapfrog kick then drift: v += a dt_kick; x += v dt_drift
__global__ void k_kick_drift(int64_t n3, double* __restrict__ x, double* __restrict__ v,
                             const double* __restrict__ a, double dt_kick, double dt_drift) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n3;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double ak = a[k] * dt_kick;
        const double vk = v[k] + ak;
        v[k] = vk;
        const double dx = vk * dt_drift;
        x[k] = x[k] + dx;
    }
}

// ---------------------------------------------------------------------------
// Eq. 6 predictor, closed form a0 + j (t - t0)
// ---------------------------------------------------------------------------
__global__ void k_predict(int64_t n, const uint8_t* __restrict__ mask, const double* __restrict__ a0,
                          const double* __restrict__ j, const double* __restrict__ t0, double t,
                          double* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (mask && !mask[i]) continue;
        if (!j) {   // no predictor: the force of the last evaluation
#pragma unroll
            for (int c = 0; c < 3; ++c) out[3 * i + c] = a0[3 * i + c];
            continue;
        }
        double dt = t - t0[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double jd = j[3 * i + c] * dt;
            out[3 * i + c] = a0[3 * i + c] + jd;
        }
    }
}

// The same with t - t0 taken from the force-age counter of Eq. 3: a row's
// counter holds the ticks since its last force update, so t - t0 = age * tick
// (exact: an integer times a power of two).
__global__ void k_predict_age(int64_t n, const uint8_t* __restrict__ mask, const double* __restrict__ a0,
                              const double* __restrict__ j, const int64_t* __restrict__ age, double tick,
                              double* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (mask && !mask[i]) continue;
        if (!j) {
#pragma unroll
            for (int c = 0; c < 3; ++c) out[3 * i + c] = a0[3 * i + c];
            continue;
        }
        double dt = (double)age[i] * tick;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double jd = j[3 * i + c] * dt;
            out[3 * i + c] = a0[3 * i + c] + jd;
        }
    }
}

// ---------------------------------------------------------------------------
// Polynomial predictor (Sec. 2.2): a log of each row's last `depth` fresh
// forces, slot-major (slot 0 newest): hist_a (depth, n, 3), hist_t (depth, n)
// ---------------------------------------------------------------------------
__global__ void k_force_log(int64_t n_rows, const int64_t* __restrict__ n_dev, const int32_t* __restrict__ idx,
                            int64_t n, int depth, const double* __restrict__ a0, double t, double* __restrict__ ha,
                            double* __restrict__ ht, int32_t* __restrict__ hn, int32_t* __restrict__ flags) {
    if (n_dev) {   // the count on the device (outside [0, n_rows]: flag, none)
        const int64_t v = *n_dev;
        const bool bad = v < 0 || v > n_rows;
        if (bad && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, AGF_BADINDEX);
        n_rows = bad ? 0 : v;
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_rows;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = idx ? (int64_t)idx[k] : k;
        if (r < 0 || r >= n) {
            atomicOr(flags, AGF_BADINDEX);
            continue;
        }
        for (int s = depth - 1; s > 0; --s) {
            ht[s * n + r] = ht[(s - 1) * n + r];
#pragma unroll
            for (int c = 0; c < 3; ++c) ha[3 * (s * n + r) + c] = ha[3 * ((s - 1) * n + r) + c];
        }
        ht[r] = t;
#pragma unroll
        for (int c = 0; c < 3; ++c) ha[3 * r + c] = a0[3 * r + c];
        const int cnt = hn[r] + 1;
        hn[r] = cnt < depth ? cnt : depth;
    }
}

// g(t) = sum_k g_k prod_{m != k} (t - t_m) / (t_k - t_m) over the newest
// logged forces: at most order + 1 of them, as many as the row has, and only
// while each is strictly older than the one before (distinct nodes).  Rows
// with nothing logged, or masked out, are left untouched.
__global__ void k_predict_poly(int64_t n, const uint8_t* __restrict__ mask, int depth, int order,
                               const double* __restrict__ ha, const double* __restrict__ ht,
                               const int32_t* __restrict__ hn, double t, double* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (mask && !mask[i]) continue;
        int cnt = hn[i];
        cnt = cnt < depth ? cnt : depth;
        if (cnt <= 0) continue;
        double tk[AG_PRED_MAX_DEPTH];
        tk[0] = ht[i];
        int nodes = 1;
        for (int k = 1; k < cnt && k <= order; ++k) {
            const double tt = ht[k * n + i];
            if (!(tt < tk[k - 1])) break;
            tk[k] = tt;
            nodes = k + 1;
        }
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < nodes; ++k) {
            double w = 1.0;
            for (int m = 0; m < nodes; ++m)
                if (m != k) w = w * ((t - tk[m]) / (tk[k] - tk[m]));
            const double* a = ha + 3 * (k * n + i);
            s0 = s0 + w * a[0];
            s1 = s1 + w * a[1];
            s2 = s2 + w * a[2];
        }
        out[3 * i] = s0;
        out[3 * i + 1] = s1;
        out[3 * i + 2] = s2;
    }
}

// ---------------------------------------------------------------------------
// device-wide exclusive scan of int32 (three passes: tile sums, scan of the
// tile sums in one block, tile scans plus offsets)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// exclusive scan of `v` across the block; returns the block total in *total
__device__ __forceinline__ int block_excl_scan(int v, int* s_w, int* total) {
    const int lane = ag_lane();
    const int wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int inc = ag_wave_incl_scan(v);
    if (lane == 63) s_w[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        int w = lane < nw ? s_w[lane] : 0;
        int wi = ag_wave_incl_scan(w);
        if (lane < nw) s_w[lane] = wi - w;
        if (lane == nw - 1) s_w[nw] = wi;
    }
    __syncthreads();
    int r = s_w[wid] + inc - v;
    *total = s_w[nw];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int32_t* __restrict__ in, int64_t n,
                                                             int32_t* __restrict__ tile_sum) {
    __shared__ int s_w[17];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    int tot;
    block_excl_scan(s, s_w, &tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_top(int32_t* __restrict__ tile_sum, int64_t ntiles,
                                                           int32_t* __restrict__ total_out) {
    __shared__ int s_w[17];
    // each thread owns a contiguous run of tiles
    int64_t per = (ntiles + kScanThreads - 1) / kScanThreads;
    int64_t lo = (int64_t)threadIdx.x * per;
    int64_t hi = lo + per < ntiles ? lo + per : ntiles;
    int s = 0;
    for (int64_t t = lo; t < hi; ++t) s += tile_sum[t];
    int tot;
    int off = block_excl_scan(s, s_w, &tot);
    for (int64_t t = lo; t < hi; ++t) {
        int v = tile_sum[t];
        tile_sum[t] = off;
        off += v;
    }
    if (threadIdx.x == 0) *total_out = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                             const int32_t* __restrict__ tile_off,
                                                             int32_t* __restrict__ out) {
    __shared__ int s_w[17];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int off = block_excl_scan(s, s_w, &tot) + tile_off[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = off;
        off += v[k];
    }
}

// Second pass of the two-launch scan: every tile first sums the totals of
// the tiles before it (at most kScanThreads * kScanTopItems of them), then
// scans its own items; the last tile writes the grand total.
constexpr int kScanTopItems = 4;

__global__ void __launch_bounds__(kScanThreads) k_scan_apply2(const int32_t* __restrict__ in, int64_t n,
                                                              const int32_t* __restrict__ tile_sum,
                                                              int32_t* __restrict__ out) {
    __shared__ int s_w[17];
    int pre = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += kScanThreads) pre += tile_sum[t];
    int pre_tot;
    block_excl_scan(pre, s_w, &pre_tot);
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int off = block_excl_scan(s, s_w, &tot) + pre_tot;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = off;
        off += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = pre_tot + tot;
}

}  // namespace

int ag_scan_i32(ag_ctx* c, const int32_t* in, int32_t* out, int64_t n) {
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles < 1) ntiles = 1;
    AG_TRY(ag_ensure(c, c->scan_tmp, (size_t)ntiles * sizeof(int32_t)));
    int32_t* ts = c->scan_tmp.as<int32_t>();
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, c->stream, in, n, ts);
    if (ntiles <= (int64_t)kScanThreads * kScanTopItems) {
        hipLaunchKernelGGL(k_scan_apply2, dim3((unsigned)ntiles), dim3(kScanThreads), 0, c->stream, in, n, ts,
                           out);
        return AG_OK;
    }
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, c->stream, ts, ntiles, out + n);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(kScanThreads), 0, c->stream, in, n, ts, out);
    return AG_OK;
}

int ag_launch_timestep(ag_ctx* c, int64_t n, const int32_t* idx, int64_t n_idx, const double* tidal,
                       double eta, double dt_max, int32_t k_max, double* dt, int8_t* bin, const int64_t* n_dev) {
    PhaseScope phase(c, AG_PHASE_STEP);
    hipLaunchKernelGGL(k_timestep, dim3(grid_for(n_idx)), dim3(kThreads), 0, c->stream, n_idx, n_dev, idx, n,
                       tidal, eta, sqrt(eta), dt_max, (int)k_max, dt, bin, c->dflags.as<int32_t>());
    return AG_OK;
}

int ag_launch_kick_drift(ag_ctx* c, int64_t n, double* x, double* v, const double* acc, double dt_kick,
                         double dt_drift) {
    PhaseScope phase(c, AG_PHASE_STEP);
    hipLaunchKernelGGL(k_kick_drift, dim3(grid_for(3 * n)), dim3(kThreads), 0, c->stream, 3 * n, x, v, acc,
                       dt_kick, dt_drift);
    return AG_OK;
}

int ag_launch_force_log(ag_ctx* c, int64_t n, const int32_t* idx, int64_t n_idx, int32_t depth,
                        const double* a0, double t, double* ha, double* ht, int32_t* hn, const int64_t* n_dev) {
    PhaseScope phase(c, AG_PHASE_STEP);
    hipLaunchKernelGGL(k_force_log, dim3(grid_for(n_idx)), dim3(kThreads), 0, c->stream, n_idx, n_dev, idx, n,
                       (int)depth, a0, t, ha, ht, hn, c->dflags.as<int32_t>());
    return AG_OK;
}

int ag_launch_predict_poly(ag_ctx* c, int64_t n, const uint8_t* mask, int32_t depth, int32_t order,
                           const double* ha, const double* ht, const int32_t* hn, double t, double* out) {
    PhaseScope phase(c, AG_PHASE_STEP);
    hipLaunchKernelGGL(k_predict_poly, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, n, mask, (int)depth,
                       (int)order, ha, ht, hn, t, out);
    return AG_OK;
}

int ag_launch_select(ag_ctx* c, int64_t n, int64_t* tf, const int8_t* bin, int64_t step_ticks,
                     int32_t tick_bin, double q_f, int32_t* active_idx, int64_t* n_active_dev,
                     double* t0, double t) {
    PhaseScope phase(c, AG_PHASE_STEP);
    AG_TRY(ag_ensure(c, c->sel_flag, (size_t)n * sizeof(int32_t)));
    AG_TRY(ag_ensure(c, c->sel_off, (size_t)(n + 1) * sizeof(int32_t)));
    int32_t* flag = c->sel_flag.as<int32_t>();
    int32_t* off = c->sel_off.as<int32_t>();
    hipLaunchKernelGGL(k_select, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, n, tf, bin, step_ticks,
                       (int)tick_bin, q_f, flag);
    AG_TRY(ag_scan_i32(c, flag, off, n));
    hipLaunchKernelGGL(k_compact, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, n, flag, off,
                       active_idx, n_active_dev, t0, t);
    return AG_OK;
}

int ag_launch_predict(ag_ctx* c, int64_t n, const uint8_t* mask, const double* a0, const double* j,
                      const double* t0, double t, double* out) {
    PhaseScope phase(c, AG_PHASE_STEP);
    hipLaunchKernelGGL(k_predict, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, n, mask, a0, j, t0, t, out);
    return AG_OK;
}

int ag_launch_predict_age(ag_ctx* c, int64_t n, const uint8_t* mask, const double* a0, const double* j,
                          const int64_t* age, double tick, double* out) {
    PhaseScope phase(c, AG_PHASE_STEP);
    hipLaunchKernelGGL(k_predict_age, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, n, mask, a0, j, age, tick,
                       out);
    return AG_OK;
}
