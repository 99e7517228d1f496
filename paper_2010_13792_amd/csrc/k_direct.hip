// k_direct.hip -- softened direct summation of g, j and T (all sources act
// on each listed target), in FP64 or with FP32 pair terms.
//
// Layout: a workgroup of eight waves owns T = 64 / Gs targets.  Each wave
// holds all T targets, Gs times over: lane l serves target l mod T in lane
// group l / T, and the 8 Gs lane groups of the workgroup each sum their own
// subset of the sources (source q of a staged tile belongs to subset
// q mod 8 Gs).  Gs (1 .. 16) is the smallest that gives enough workgroups to
// fill the chip, so a target set of a few thousand still spreads over every
// SIMD without any exchange between workgroups.  Sources are staged through
// LDS 1024 at a time (two coalesced loads per thread); the Gs groups of a
// wave read Gs neighbouring sources at once (broadcasts within each group).
// FP64 runs one workgroup per CU with up to 256 registers and takes kChains
// sources per lane at a time (independent dependency chains); FP32 pairs
// run two workgroups per CU within 128 registers, one source at a time.
// At the end the subsets are added in a fixed tree: across the lane groups
// of a wave by butterfly shuffles, then across the eight waves in LDS in
// wave order -- bit-reproducible, no scratch and no atomics.  Only a target
// set too small to fill the chip even at Gs = 16 is also split over sources
// (grid.y): each split writes its FP64 sums to scratch and a second kernel
// adds them in split order (the kernel boundary orders the two, so no
// device-wide fence is needed).
//
// The self pair is left out by a test that only the staged tiles holding one
// of the wave's own targets run.  The Newtonian f and D are formed on every
// lane; the kernel interior replaces them where some lane of the wave has a
// source inside its softening length (a wave-uniform branch).
//
// FP64 mode: every operation in FP64; 1/sqrt(r^2) from the hardware's FP64
// reciprocal square root estimate and one third-order correction (rsqrt_f64).
// FP32-pair mode: the separation d = x_j - x_i is formed in FP64 and rounded
// once to FP32 (the exact relative coordinate), the pair term is computed in
// FP32, and each lane's FP32 sum over one staged tile is folded into FP64
// accumulators.
//
// Periodic cube of side L (kPer): d is replaced by its nearest image
// d - L rint(d / L), in FP64, before anything else.
//
// Per-particle softening (kSoft): each pair's f and D are the means of the
// target's and the source's kernels (hs, input order).
#include <mutex>

#include "ag_internal.h"
#include "pair.h"

namespace {

constexpr int kWaves = 8;                // waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr int kSrc = 2 * kThreads;       // sources per staged tile
constexpr int kParts = 12;               // g (3), j (3), S (6)
constexpr int kChains = 4;                // FP64 sources per lane per iteration
constexpr int kMinTShift = 2;            // at least 4 targets per workgroup (at most 16 lane groups)

__device__ __forceinline__ double near_img(double d, double L) { return d - L * rint(d / L); }

// 1/sqrt(x), x > 0 normal: the hardware estimate y (relative error at most
// about 2^-24 over arguments spread across 40 decades, as measured on
// gfx950) corrected once by the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ...
// in e = 1 - x y^2, to second order: the relative error left is about
// (5/16) e^3, far below FP64 rounding, for five operations (two Newton steps
// take eight)
__device__ __forceinline__ double rsqrt_f64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x * y, y, 1.0);
    const double p = __builtin_fma(0.375, e, 0.5);
    return __builtin_fma(y * e, p, y);
}

template <class R>
__device__ __forceinline__ R rsqrt_any(R r2) {
    if constexpr (sizeof(R) == 8) return rsqrt_f64(r2);
    else return __builtin_amdgcn_rsqf(r2);
}

// The sums of one target: g, j and S = sum m [f I + D d d^T], whose
// diagonal term sum m f is kept once (smf) and added to the three diagonal
// entries at the end.
template <class R>
struct DirAcc {
    R ax, ay, az, jx, jy, jz, sxx, syy, szz, sxy, sxz, syz, smf;
    __device__ __forceinline__ void zero() {
        ax = ay = az = jx = jy = jz = sxx = syy = szz = sxy = sxz = syz = smf = R(0);
    }
    template <class Q>
    __device__ __forceinline__ void add(const DirAcc<Q>& B) {
        ax += B.ax; ay += B.ay; az += B.az;
        jx += B.jx; jy += B.jy; jz += B.jz;
        sxx += B.sxx; syy += B.syy; szz += B.szz;
        sxy += B.sxy; sxz += B.sxz; syz += B.syz;
        smf += B.smf;
    }
};

// one pair's terms from mf = m f and mD = m D (pair.h states the formulas)
template <class R>
__device__ __forceinline__ void pair_add(R dx, R dy, R dz, R nx, R ny, R nz, R mf, R mD, DirAcc<R>& A) {
    A.ax += mf * dx;
    A.ay += mf * dy;
    A.az += mf * dz;
    const R dn = dx * nx + dy * ny + dz * nz;
    const R s = mD * dn;
    A.jx += mf * nx + s * dx;
    A.jy += mf * ny + s * dy;
    A.jz += mf * nz + s * dz;
    const R tx = mD * dx, ty = mD * dy, tz = mD * dz;
    A.smf += mf;
    A.sxx += tx * dx;
    A.syy += ty * dy;
    A.szz += tz * dz;
    A.sxy += tx * dy;
    A.sxz += tx * dz;
    A.syz += ty * dz;
}

// The Newtonian f and D are formed for every lane; the kernel interior
// replaces them only where some lane of the wave has a source inside its
// softening length (a wave-uniform branch, rarely taken).
template <class R>
__device__ __forceinline__ void pair_any(R dx, R dy, R dz, R nx, R ny, R nz, R mj, R h2, R hinv, DirAcc<R>& A) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ri = rsqrt_any<R>(r2);
    const R ri2 = ri * ri;
    R mf = mj * (ri * ri2);
    R mD = mf * (R(-3) * ri2);   // m D = m f (-3 / r^2) outside the kernel
    if (__ballot(r2 < h2) != 0) {
        if (r2 < h2) {
            R f, D;
            spline_fd<R>(r2, hinv, f, D);
            mf = mj * f;
            mD = mj * D;
        }
    }
    pair_add<R>(dx, dy, dz, nx, ny, nz, mf, mD, A);
}

// per-particle softening: f and D are the means of the target's and the
// source's kernels, each Newtonian beyond its own length
template <class R>
__device__ __forceinline__ void pair_soft(R dx, R dy, R dz, R nx, R ny, R nz, R mj, R hi_, R hj, DirAcc<R>& A) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    const R ri = rsqrt_any<R>(r2);
    const R ri2 = ri * ri;
    const R fN = ri * ri2;
    const R DN = R(-3) * fN * ri2;
    R fs[2] = {fN, fN}, Ds[2] = {DN, DN};
    const R hs[2] = {hi_, hj};
#pragma unroll
    for (int k = 0; k < 2; ++k)
        if (r2 < hs[k] * hs[k]) spline_fd<R>(r2, R(1) / hs[k], fs[k], Ds[k]);
    pair_add<R>(dx, dy, dz, nx, ny, nz, mj * (R(0.5) * (fs[0] + fs[1])), mj * (R(0.5) * (Ds[0] + Ds[1])), A);
}

struct DirectArgs {
    int64_t n;
    const double* x;
    const double* v;
    const double* m;
    const double* hs;        // per-particle softening lengths (kSoft)
    const int32_t* idx;      // listed rows (null: 0 .. n_act)
    int64_t n_act;
    double h, L, G;
    int tshift;              // log2 of the targets per workgroup T (T = 64 / Gs)
    int64_t chunk;           // sources per split
    int nsplit;
    double* part;            // [tile][split][component][T] FP64 sums (nsplit > 1)
    double* acc;
    double* jerk;
    double* tidal;
    int32_t* flags;
};

union DirectLds {
    struct {
        double x[kSrc], y[kSrc], z[kSrc], m[kSrc];
        double vx[kSrc], vy[kSrc], vz[kSrc];
        double h[kSrc];
    } src;
    double red[kWaves][kParts][64];   // each wave's sums per target, added in wave order
};

// the separation and relative velocity of staged source q from the target
template <bool kPer>
__device__ __forceinline__ void sep_at(const DirectLds& S, const DirectArgs& P, int q, double xi, double yi, double zi,
                                       double vxi, double vyi, double vzi, double& dx, double& dy, double& dz,
                                       double& nx, double& ny, double& nz) {
    dx = S.src.x[q] - xi;
    dy = S.src.y[q] - yi;
    dz = S.src.z[q] - zi;
    if (kPer) {
        dx = near_img(dx, P.L);
        dy = near_img(dy, P.L);
        dz = near_img(dz, P.L);
    }
    nx = S.src.vx[q] - vxi;
    ny = S.src.vy[q] - vyi;
    nz = S.src.vz[q] - vzi;
}

// a lane's share of one staged tile of cnt sources: q = q0, q0 + stride, ...;
// with kExcl the source at tile slot qs (the lane's own target) is left out.
// FP64 pair terms; without per-particle softening kChains sources at a time
// (independent dependency chains: the FP64 launch runs two waves per SIMD).
template <bool kPer, bool kSoft, bool kExcl>
__device__ __forceinline__ void pairs_tile(const DirectLds& S, const DirectArgs& P, int q0, int stride, int cnt,
                                           int qs, double xi, double yi, double zi, double vxi, double vyi,
                                           double vzi, double hi_, double h2, double hinv, DirAcc<double>& A) {
    int q = q0;
    if constexpr (!kSoft && kChains > 1) {
        constexpr int C = kChains;
        for (; q + (C - 1) * stride < cnt; q += C * stride) {
            double dx[C], dy[C], dz[C], nx[C], ny[C], nz[C], r2[C], mf[C], mD[C], mj[C];
            bool inside = false;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int qc = q + c * stride;
                sep_at<kPer>(S, P, qc, xi, yi, zi, vxi, vyi, vzi, dx[c], dy[c], dz[c], nx[c], ny[c], nz[c]);
                mj[c] = (kExcl && qc == qs) ? 0.0 : S.src.m[qc];
                r2[c] = dx[c] * dx[c] + dy[c] * dy[c] + dz[c] * dz[c];
                inside = inside || r2[c] < h2;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double ri = rsqrt_f64(r2[c]);
                const double ri2 = ri * ri;
                mf[c] = mj[c] * (ri * ri2);
                mD[c] = mf[c] * (-3.0 * ri2);
            }
            if (__ballot(inside) != 0) {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (r2[c] < h2) {
                        double f, D;
                        spline_fd<double>(r2[c], hinv, f, D);
                        mf[c] = mj[c] * f;
                        mD[c] = mj[c] * D;
                    }
            }
#pragma unroll
            for (int c = 0; c < C; ++c) pair_add<double>(dx[c], dy[c], dz[c], nx[c], ny[c], nz[c], mf[c], mD[c], A);
        }
    }
    for (; q < cnt; q += stride) {
        double dx, dy, dz, nx, ny, nz;
        sep_at<kPer>(S, P, q, xi, yi, zi, vxi, vyi, vzi, dx, dy, dz, nx, ny, nz);
        const double mj = (kExcl && q == qs) ? 0.0 : S.src.m[q];
        if (kSoft) pair_soft<double>(dx, dy, dz, nx, ny, nz, mj, hi_, S.src.h[q], A);
        else pair_any<double>(dx, dy, dz, nx, ny, nz, mj, h2, hinv, A);
    }
}

// the same with FP32 pair terms on the FP64 separations rounded once
template <bool kPer, bool kSoft, bool kExcl>
__device__ __forceinline__ void pairs_tile_f32(const DirectLds& S, const DirectArgs& P, int q0, int stride, int cnt,
                                               int qs, double xi, double yi, double zi, double vxi, double vyi,
                                               double vzi, double hi_, float h2f, float hinvf, DirAcc<float>& B) {
    for (int q = q0; q < cnt; q += stride) {
        double dx, dy, dz, nx, ny, nz;
        sep_at<kPer>(S, P, q, xi, yi, zi, vxi, vyi, vzi, dx, dy, dz, nx, ny, nz);
        const float mj = (kExcl && q == qs) ? 0.0f : (float)S.src.m[q];
        if (kSoft)
            pair_soft<float>((float)dx, (float)dy, (float)dz, (float)nx, (float)ny, (float)nz, mj, (float)hi_,
                             (float)S.src.h[q], B);
        else
            pair_any<float>((float)dx, (float)dy, (float)dz, (float)nx, (float)ny, (float)nz, mj, h2f, hinvf, B);
    }
}

// one target row's outputs from its FP64 sums (component c of 12)
__device__ __forceinline__ void write_row(const DirectArgs& P, int64_t r, int c, double sum) {
    if (c < 3) {
        if (P.acc) P.acc[3 * r + c] = P.G * sum;
    } else if (c < 6) {
        if (P.jerk) P.jerk[3 * r + c - 3] = P.G * sum;
    } else if (P.tidal) {
        P.tidal[6 * r + c - 6] = -P.G * sum;
    }
}

// the row of listed target k, or -1 (past the list, or a bad index: flagged)
__device__ __forceinline__ int64_t target_row(const DirectArgs& P, int64_t k, bool flag) {
    if (k >= P.n_act) return -1;
    const int64_t i = P.idx ? (int64_t)P.idx[k] : k;
    if (i < 0 || i >= P.n) {
        if (flag) atomicOr(P.flags, AGF_BADINDEX);
        return -1;
    }
    return i;
}

template <bool kFP64, bool kPer, bool kSoft>
__device__ __forceinline__ void direct_body(DirectLds& S, const DirectArgs& P) {
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int T = 1 << P.tshift;               // targets per workgroup
    const int Gs = 64 >> P.tshift;             // lane groups per wave
    const int t = lane & (T - 1);
    const int sub = w * Gs + (lane >> P.tshift);   // this lane's source subset
    const int nsub = kWaves * Gs;
    const int64_t i = target_row(P, (int64_t)blockIdx.x * T + t, lane < T && w == 0);
    double xi = 0, yi = 0, zi = 0, vxi = 0, vyi = 0, vzi = 0, hi_ = 1.0;
    if (i >= 0) {
        xi = P.x[3 * i]; yi = P.x[3 * i + 1]; zi = P.x[3 * i + 2];
        vxi = P.v[3 * i]; vyi = P.v[3 * i + 1]; vzi = P.v[3 * i + 2];
        if (kSoft) hi_ = P.hs[i];
    }
    const int64_t j0 = (int64_t)blockIdx.y * P.chunk;
    const int64_t j1 = j0 + P.chunk < P.n ? j0 + P.chunk : P.n;

    DirAcc<double> A;
    A.zero();
    const double h2 = P.h * P.h, hinv = 1.0 / P.h;
    const float h2f = (float)h2, hinvf = (float)hinv;
    for (int64_t t0 = j0; t0 < j1; t0 += kSrc) {
        __syncthreads();
#pragma unroll
        for (int u = threadIdx.x; u < kSrc; u += kThreads) {
            const int64_t js = t0 + u;
            if (js < j1) {
                S.src.x[u] = P.x[3 * js];
                S.src.y[u] = P.x[3 * js + 1];
                S.src.z[u] = P.x[3 * js + 2];
                S.src.m[u] = P.m[js];
                S.src.vx[u] = P.v[3 * js];
                S.src.vy[u] = P.v[3 * js + 1];
                S.src.vz[u] = P.v[3 * js + 2];
                if (kSoft) S.src.h[u] = P.hs[js];
            }
        }
        __syncthreads();
        const int cnt = (int)((j1 - t0) < kSrc ? (j1 - t0) : kSrc);
        // the self pair is left out: only the tiles that hold one of the
        // wave's own targets pay for the test
        const bool self_here = __ballot(i >= t0 && i < t0 + cnt) != 0;
        if (i < 0) continue;
        const int qs = (i >= t0 && i < t0 + cnt) ? (int)(i - t0) : -1;   // -1 never matches
        if (kFP64) {
            if (self_here) pairs_tile<kPer, kSoft, true>(S, P, sub, nsub, cnt, qs, xi, yi, zi, vxi, vyi, vzi, hi_, h2, hinv, A);
            else pairs_tile<kPer, kSoft, false>(S, P, sub, nsub, cnt, qs, xi, yi, zi, vxi, vyi, vzi, hi_, h2, hinv, A);
        } else {
            DirAcc<float> B;
            B.zero();
            if (self_here)
                pairs_tile_f32<kPer, kSoft, true>(S, P, sub, nsub, cnt, qs, xi, yi, zi, vxi, vyi, vzi, hi_, h2f, hinvf, B);
            else
                pairs_tile_f32<kPer, kSoft, false>(S, P, sub, nsub, cnt, qs, xi, yi, zi, vxi, vyi, vzi, hi_, h2f, hinvf, B);
            A.add(B);
        }
    }
    // the Gs lane groups of the wave: a butterfly over lane offsets T, 2T, ...
    // (every lane of a target ends with the same tree sum)
    double vals[kParts] = {A.ax,         A.ay,         A.az,         A.jx,  A.jy,  A.jz,
                           A.smf + A.sxx, A.smf + A.syy, A.smf + A.szz, A.sxy, A.sxz, A.syz};
    for (int off = T; off < 64; off <<= 1) {
#pragma unroll
        for (int c = 0; c < kParts; ++c) vals[c] += __shfl_xor(vals[c], off);
    }
    __syncthreads();   // every wave is done with the staged sources
    if (lane < T) {
#pragma unroll
        for (int c = 0; c < kParts; ++c) S.red[w][c][lane] = vals[c];
    }
    __syncthreads();
    // the eight waves, added in wave order: one thread per (component, target)
    const int64_t tile = blockIdx.x;
    for (int e = threadIdx.x; e < kParts * T; e += kThreads) {
        const int c = e >> P.tshift, tt = e & (T - 1);
        double sum = S.red[0][c][tt];
#pragma unroll
        for (int ww = 1; ww < kWaves; ++ww) sum += S.red[ww][c][tt];
        if (P.nsplit == 1) {
            const int64_t r = target_row(P, tile * T + tt, false);
            if (r >= 0) write_row(P, r, c, sum);
        } else {
            P.part[((tile * P.nsplit + blockIdx.y) * kParts + c) * T + tt] = sum;
        }
    }
}

// FP64: one workgroup per CU (kBlocks64), up to 256 registers for the
// chains of kChains pairs; FP32 pairs: two workgroups per CU (kBlocks32), at
// most 128 registers
template <bool kPer, bool kSoft>
__global__ void __launch_bounds__(kThreads) k_direct64(DirectArgs P) {
    __shared__ DirectLds S;
    direct_body<true, kPer, kSoft>(S, P);
}
template <bool kPer, bool kSoft>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) k_direct32(DirectArgs P) {
    __shared__ DirectLds S;
    direct_body<false, kPer, kSoft>(S, P);
}

// the splits of each target tile added in split order (a split launch only)
__global__ void __launch_bounds__(256) k_direct_splits(DirectArgs P, int64_t tiles) {
    const int T = 1 << P.tshift;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (tile, component, target)
    if (e >= tiles * kParts * T) return;
    const int64_t tile = e / (kParts * T);
    const int c = (int)((e / T) % kParts), tt = (int)(e & (T - 1));
    const double* p = P.part + (tile * P.nsplit * kParts + c) * T + tt;
    double sum = 0.0;
    for (int q = 0; q < P.nsplit; ++q) sum += p[(int64_t)q * kParts * T];
    const int64_t r = target_row(P, tile * T + tt, false);
    if (r >= 0) write_row(P, r, c, sum);
}

}  // namespace

// Launch shape: the fewest lane groups per wave Gs (1 .. 16) that give at
// least `blocks` workgroups (kBlocks64 = one per CU for FP64, kBlocks32 = two
// per CU for FP32 pairs); only below that at Gs = 16 is the source range
// split as well (grid.y), so that tiles x splits stays below 2 blocks.  Each
// split covers a multiple of the 8 Gs subsets.
constexpr int64_t kBlocks64 = 256;
constexpr int64_t kBlocks32 = 512;
constexpr int64_t kDirectBlocks = kBlocks64 > kBlocks32 ? kBlocks64 : kBlocks32;   // bounds the split scratch

void ag_direct_shape(int64_t n, int64_t n_act, int precision, int* tshift, int64_t* tiles, int64_t* nsplit,
                     int64_t* chunk) {
    const int64_t blocks = precision == AG_FP64 ? kBlocks64 : kBlocks32;
    int ts = 6;
    int64_t t = (n_act + 63) >> 6;
    while (ts > kMinTShift && t < blocks) {
        --ts;
        t = (n_act + (1 << ts) - 1) >> ts;
    }
    const int64_t nsub = (int64_t)kWaves * (64 >> ts);
    int64_t s = 1;
    if (t < blocks) {
        s = (blocks + t - 1) / t;
        const int64_t max_split = (n + nsub - 1) / nsub;
        if (s > max_split) s = max_split;
        if (s > 65535) s = 65535;
        if (s < 1) s = 1;
    }
    int64_t c = (n + s - 1) / s;
    c = (c + nsub - 1) / nsub * nsub;
    *tshift = ts;
    *tiles = t;
    *nsplit = (n + c - 1) / c;
    *chunk = c;
}

size_t ag_direct_scratch_bytes(int64_t n, int64_t n_act, int precision) {
    int ts;
    int64_t t, s, c;
    ag_direct_shape(n, n_act, precision, &ts, &t, &s, &c);
    if (s <= 1) return 0;
    return (size_t)t * s * kParts * ((size_t)1 << ts) * sizeof(double);
}

int ag_launch_direct(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                     const int32_t* idx, int64_t n_act, double eps, double G, int precision,
                     double* acc, double* jerk, double* tidal, void* scratch, bool timed) {
    int tshift;
    int64_t tiles, nsplit, chunk;
    ag_direct_shape(n, n_act, precision, &tshift, &tiles, &nsplit, &chunk);
    DirectArgs P{};
    P.n = n;
    P.x = x;
    P.v = v;
    P.m = m;
    P.hs = c->soft_n > 0 ? c->soft_h.as<double>() : nullptr;
    P.idx = idx;
    P.n_act = n_act;
    P.h = eps;
    P.L = c->box;
    P.G = G;
    P.tshift = tshift;
    P.chunk = chunk;
    P.nsplit = (int)nsplit;
    P.part = nsplit > 1 ? reinterpret_cast<double*>(scratch) : nullptr;
    P.acc = acc;
    P.jerk = jerk;
    P.tidal = tidal;
    P.flags = c->dflags.as<int32_t>();
    PhaseScope phase(c, timed ? AG_PHASE_DIRECT : -1);
    dim3 grid((unsigned)tiles, (unsigned)nsplit);
    hipStream_t st = c->stream;
    const bool fp64 = precision == AG_FP64, per = P.L > 0.0, soft = P.hs != nullptr;
#define AG_DIRECT(K, B, C) hipLaunchKernelGGL((K<B, C>), grid, dim3(kThreads), 0, st, P)
    if (fp64) {
        if (per) { if (soft) AG_DIRECT(k_direct64, true, true); else AG_DIRECT(k_direct64, true, false); }
        else { if (soft) AG_DIRECT(k_direct64, false, true); else AG_DIRECT(k_direct64, false, false); }
    } else {
        if (per) { if (soft) AG_DIRECT(k_direct32, true, true); else AG_DIRECT(k_direct32, true, false); }
        else { if (soft) AG_DIRECT(k_direct32, false, true); else AG_DIRECT(k_direct32, false, false); }
    }
#undef AG_DIRECT
    if (nsplit > 1) {
        const int64_t work = tiles * kParts * ((int64_t)1 << tshift);
        hipLaunchKernelGGL(k_direct_splits, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, P, tiles);
    }
    return AG_OK;
}

// ---------------------------------------------------------------------------
// The allocation-free direct sum, for callers that cannot allocate device
// memory: the split sums live in a file-scope device array of fixed size.
// The launch shape bounds the scratch for every size (a split happens only
// with fewer target tiles of 4 than the precision's workgroup count, at most
// kDirectBlocks, so tiles x splits < 2 kDirectBlocks), so no call is refused
// for its size.  Every call on a
// device shares that device's copy of the array: calls that overlap on one
// device race.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocBytes = (size_t)(2 * kDirectBlocks) * kParts * 4 * sizeof(double);
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // the array's address on each device
}  // namespace

int ag_direct_noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return ag_fail(AG_EINVAL, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return AG_OK;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return ag_fail(AG_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return AG_OK;
}

extern "C" int ag_grav_direct_noalloc(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                                      const int32_t* idx, int64_t n_act, double eps, double G, int precision,
                                      double* acc, double* jerk, double* tidal) {
    AG_TRY(ag_direct_check(c, n, x, v, m, idx, n_act, eps, G, precision));
    if (n_act == 0) return AG_OK;
    const size_t bytes = ag_direct_scratch_bytes(n, n_act, precision);
    if (bytes > kNoAllocBytes)
        return ag_fail(AG_EINVAL, "the direct sum needs %zu bytes of scratch, above the %zu this entry point holds",
                       bytes, kNoAllocBytes);
    void* p = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = c->device < kMaxDevices ? g_scratch_ptr[c->device] : nullptr;
    }
    if (!p) return ag_fail(AG_ESTATE, "no direct-sum scratch on device %d", c->device);
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_direct(c, n, x, v, m, idx, n_act, eps, G, precision, acc, jerk, tidal, bytes > 0 ? p : nullptr,
                            false));
    return ag_check_launch("grav direct (no allocation)");
}
