// k_direct.hip -- softened direct summation of g, j and T (all sources act
// on each listed target), in FP64 or with FP32 pair terms.
//
// Layout: a workgroup of four waves owns 64 targets (one per lane, the same
// 64 in every wave) and one contiguous chunk of sources.  The chunk is
// staged through LDS 256 sources at a time (one coalesced load per thread);
// wave w sums sources w, w + 4, ... of every staged tile, reading them as LDS
// broadcasts, so the four waves of a workgroup interleave their pair chains
// on the SIMDs of one CU.  At the end the four waves' sums are added in LDS
// in a fixed order.  The self pair is left out by a test that only the
// tiles holding one of the wave's own targets run.  The Newtonian f and D
// are formed on every lane; the kernel interior replaces them where some
// lane of the wave has a source inside its softening length (a
// wave-uniform branch).  A small target set is split over sources (grid.y) so
// the launch holds enough workgroups to fill the 256 CUs; each split writes
// its FP64 sums to scratch, and the last split of a target tile to finish
// (an agent-scope counter per tile) adds all splits in split order and
// writes the rows -- one launch, bit-reproducible, and the counter is back
// at zero afterwards.
//
// FP64 mode: every operation in FP64; 1/sqrt(r^2) from the hardware's FP64
// reciprocal square root estimate refined by two Newton steps.
// FP32-pair mode: the separation d = x_j - x_i is formed in FP64 and rounded
// once to FP32 (the exact relative coordinate), the pair term is computed in
// FP32, and each wave's FP32 sum over one staged tile is folded into FP64
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

constexpr int kTile = 64;        // targets per workgroup (one per lane)
constexpr int kWaves = 4;        // waves per workgroup, each on a quarter of every source tile
constexpr int kThreads = kTile * kWaves;
constexpr int kSrc = kThreads;   // sources per staged tile
constexpr int kParts = 12;       // g (3), j (3), S (6)

__device__ __forceinline__ double near_img(double d, double L) { return d - L * rint(d / L); }

// 1/sqrt(x), x > 0 normal: the hardware estimate plus two Newton steps
// y <- y (3 - x y^2) / 2 (each step squares the relative error)
__device__ __forceinline__ double rsqrt_f64(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double e = __builtin_fma(-x * y, y, 1.0);
        y = __builtin_fma(0.5 * y, e, y);
    }
    return y;
}

// The pair term of pair.h with the reciprocal square roots above.  The
// Newtonian f and D are formed for every lane; the kernel interior replaces
// them only where some lane of the wave has a source inside its softening
// length (a wave-uniform branch, rarely taken).
template <class R>
__device__ __forceinline__ void pair_any(R dx, R dy, R dz, R nx, R ny, R nz, R mj, R h2, R hinv, PairAcc<R>& A) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    R ri;
    if constexpr (sizeof(R) == 8) ri = rsqrt_f64(r2);
    else ri = __builtin_amdgcn_rsqf(r2);
    const R ri2 = ri * ri;
    R f = ri * ri2;
    R D = R(-3) * f * ri2;
    if (__ballot(r2 < h2) != 0) {
        if (r2 < h2) spline_fd<R>(r2, hinv, f, D);
    }
    const R mf = mj * f;
    const R mD = mj * D;
    A.ax += mf * dx;
    A.ay += mf * dy;
    A.az += mf * dz;
    const R dn = dx * nx + dy * ny + dz * nz;
    const R s = mD * dn;
    A.jx += mf * nx + s * dx;
    A.jy += mf * ny + s * dy;
    A.jz += mf * nz + s * dz;
    const R tx = mD * dx, ty = mD * dy, tz = mD * dz;
    A.sxx += mf + tx * dx;
    A.syy += mf + ty * dy;
    A.szz += mf + tz * dz;
    A.sxy += tx * dy;
    A.sxz += tx * dz;
    A.syz += ty * dz;
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
    int64_t chunk;           // sources per split (a multiple of kSrc)
    int nsplit;
    double* part;            // [tile][split][component][lane] FP64 sums (nsplit > 1)
    uint32_t* count;         // [tile] splits finished (nsplit > 1), zero between calls
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
    double red[kWaves - 1][kParts][kTile];   // waves 1..3 hand their sums to wave 0
};

// wave w's share of one staged tile of cnt sources: FP64 pair terms; with
// kExcl the source at tile slot qs (the target itself) is left out
template <bool kPer, bool kSoft, bool kExcl>
__device__ __forceinline__ void pair_at(const DirectLds& S, const DirectArgs& P, int q, int qs, double xi, double yi,
                                        double zi, double vxi, double vyi, double vzi, double hi_, double h2,
                                        double hinv, PairAcc<double>& A) {
    const double mj = (kExcl && q == qs) ? 0.0 : S.src.m[q];
    double dx = S.src.x[q] - xi, dy = S.src.y[q] - yi, dz = S.src.z[q] - zi;
    if (kPer) {
        dx = near_img(dx, P.L);
        dy = near_img(dy, P.L);
        dz = near_img(dz, P.L);
    }
    const double nx = S.src.vx[q] - vxi, ny = S.src.vy[q] - vyi, nz = S.src.vz[q] - vzi;
    if (kSoft) pair_interact_soft<double>(dx, dy, dz, nx, ny, nz, mj, hi_, S.src.h[q], A);
    else pair_any<double>(dx, dy, dz, nx, ny, nz, mj, h2, hinv, A);
}

template <bool kPer, bool kSoft, bool kExcl>
__device__ __forceinline__ void pairs_tile(const DirectLds& S, const DirectArgs& P, int w, int cnt, int qs, double xi,
                                           double yi, double zi, double vxi, double vyi, double vzi, double hi_,
                                           double h2, double hinv, PairAcc<double>& A) {
    for (int q = w; q < cnt; q += kWaves)
        pair_at<kPer, kSoft, kExcl>(S, P, q, qs, xi, yi, zi, vxi, vyi, vzi, hi_, h2, hinv, A);
}

// the same with FP32 pair terms on the FP64 separations rounded once
template <bool kPer, bool kSoft, bool kExcl>
__device__ __forceinline__ void pairs_tile_f32(const DirectLds& S, const DirectArgs& P, int w, int cnt, int qs,
                                               double xi, double yi, double zi, double vxi, double vyi, double vzi,
                                               double hi_, float h2f, float hinvf, PairAcc<float>& B) {
    for (int q = w; q < cnt; q += kWaves) {
        const float mj = (kExcl && q == qs) ? 0.0f : (float)S.src.m[q];
        double dx = S.src.x[q] - xi, dy = S.src.y[q] - yi, dz = S.src.z[q] - zi;
        if (kPer) {
            dx = near_img(dx, P.L);
            dy = near_img(dy, P.L);
            dz = near_img(dz, P.L);
        }
        const float nx = (float)(S.src.vx[q] - vxi), ny = (float)(S.src.vy[q] - vyi), nz = (float)(S.src.vz[q] - vzi);
        if (kSoft)
            pair_interact_soft<float>((float)dx, (float)dy, (float)dz, nx, ny, nz, mj, (float)hi_, (float)S.src.h[q],
                                      B);
        else
            pair_any<float>((float)dx, (float)dy, (float)dz, nx, ny, nz, mj, h2f, hinvf, B);
    }
}

template <bool kFP64, bool kPer, bool kSoft>
__global__ void __launch_bounds__(kThreads) k_direct(DirectArgs P) {
    __shared__ DirectLds S;
    __shared__ bool s_last;
    const int lane = threadIdx.x & (kTile - 1);
    const int w = threadIdx.x / kTile;
    const int64_t k = (int64_t)blockIdx.x * kTile + lane;
    const bool live = k < P.n_act;
    int64_t i = -1;
    if (live) {
        i = P.idx ? (int64_t)P.idx[k] : k;
        if (i < 0 || i >= P.n) {
            if (w == 0) atomicOr(P.flags, AGF_BADINDEX);
            i = -1;
        }
    }
    double xi = 0, yi = 0, zi = 0, vxi = 0, vyi = 0, vzi = 0, hi_ = 1.0;
    if (i >= 0) {
        xi = P.x[3 * i]; yi = P.x[3 * i + 1]; zi = P.x[3 * i + 2];
        vxi = P.v[3 * i]; vyi = P.v[3 * i + 1]; vzi = P.v[3 * i + 2];
        if (kSoft) hi_ = P.hs[i];
    }
    const int64_t j0 = (int64_t)blockIdx.y * P.chunk;
    const int64_t j1 = j0 + P.chunk < P.n ? j0 + P.chunk : P.n;

    PairAcc<double> A;
    A.zero();
    const double h2 = P.h * P.h, hinv = 1.0 / P.h;
    const float h2f = (float)h2, hinvf = (float)hinv;

    for (int64_t t0 = j0; t0 < j1; t0 += kSrc) {
        const int64_t js = t0 + threadIdx.x;
        __syncthreads();
        if (js < j1) {
            S.src.x[threadIdx.x] = P.x[3 * js];
            S.src.y[threadIdx.x] = P.x[3 * js + 1];
            S.src.z[threadIdx.x] = P.x[3 * js + 2];
            S.src.m[threadIdx.x] = P.m[js];
            S.src.vx[threadIdx.x] = P.v[3 * js];
            S.src.vy[threadIdx.x] = P.v[3 * js + 1];
            S.src.vz[threadIdx.x] = P.v[3 * js + 2];
            if (kSoft) S.src.h[threadIdx.x] = P.hs[js];
        }
        __syncthreads();
        const int cnt = (int)((j1 - t0) < kSrc ? (j1 - t0) : kSrc);
        // the self pair is left out: only the tiles that hold one of the
        // wave's own targets (one tile in n / 256 when every row is listed)
        // pay for the test
        const bool self_here = __ballot(i >= t0 && i < t0 + cnt) != 0;
        if (i < 0) continue;
        const int qs = self_here ? (int)(i - t0) : -1;   // -1 never matches
        if (kFP64) {
            if (self_here) pairs_tile<kPer, kSoft, true>(S, P, w, cnt, qs, xi, yi, zi, vxi, vyi, vzi, hi_, h2, hinv, A);
            else pairs_tile<kPer, kSoft, false>(S, P, w, cnt, qs, xi, yi, zi, vxi, vyi, vzi, hi_, h2, hinv, A);
        } else {
            PairAcc<float> B;
            B.zero();
            if (self_here)
                pairs_tile_f32<kPer, kSoft, true>(S, P, w, cnt, qs, xi, yi, zi, vxi, vyi, vzi, hi_, h2f, hinvf, B);
            else
                pairs_tile_f32<kPer, kSoft, false>(S, P, w, cnt, qs, xi, yi, zi, vxi, vyi, vzi, hi_, h2f, hinvf, B);
            A.ax += B.ax; A.ay += B.ay; A.az += B.az;
            A.jx += B.jx; A.jy += B.jy; A.jz += B.jz;
            A.sxx += B.sxx; A.syy += B.syy; A.szz += B.szz;
            A.sxy += B.sxy; A.sxz += B.sxz; A.syz += B.syz;
        }
    }
    // the four waves' sums, added in wave order by wave 0
    double vals[kParts] = {A.ax, A.ay, A.az, A.jx, A.jy, A.jz, A.sxx, A.syy, A.szz, A.sxy, A.sxz, A.syz};
    __syncthreads();   // every wave is done with the staged sources
    if (w > 0) {
#pragma unroll
        for (int c = 0; c < kParts; ++c) S.red[w - 1][c][lane] = vals[c];
    }
    __syncthreads();
    const int64_t tile = blockIdx.x;
    if (w == 0) {
#pragma unroll
        for (int c = 0; c < kParts; ++c)
            vals[c] = (vals[c] + S.red[0][c][lane]) + (S.red[1][c][lane] + S.red[2][c][lane]);
        if (P.nsplit == 1) {
            if (i >= 0) {
                if (P.acc) {
                    P.acc[3 * i] = P.G * vals[0]; P.acc[3 * i + 1] = P.G * vals[1]; P.acc[3 * i + 2] = P.G * vals[2];
                }
                if (P.jerk) {
                    P.jerk[3 * i] = P.G * vals[3]; P.jerk[3 * i + 1] = P.G * vals[4]; P.jerk[3 * i + 2] = P.G * vals[5];
                }
                if (P.tidal) {
#pragma unroll
                    for (int c = 0; c < 6; ++c) P.tidal[6 * i + c] = -P.G * vals[6 + c];
                }
            }
            return;
        }
        double* p = P.part + ((tile * P.nsplit + blockIdx.y) * kParts) * kTile + lane;
#pragma unroll
        for (int c = 0; c < kParts; ++c) p[c * kTile] = vals[c];
    }
    if (P.nsplit == 1) return;
    // the last split of this tile to finish adds them all, in split order
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t done =
            __hip_atomic_fetch_add(P.count + tile, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = done == (uint32_t)(P.nsplit - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // (every thread) see the other splits' sums
    // every thread adds the splits of three (component, target) entries in
    // split order, its loads issued eight splits at a time
    const double* base = P.part + tile * P.nsplit * (kParts * kTile);
    for (int e = threadIdx.x; e < kParts * kTile; e += kThreads) {
        const int c = e / kTile, l = e % kTile;
        double sum = 0.0;
        int q = 0;
        for (; q + 8 <= P.nsplit; q += 8) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = base[(q + u) * (kParts * kTile) + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) sum += t[u];
        }
        for (; q < P.nsplit; ++q) sum += base[q * (kParts * kTile) + e];
        const int64_t kk = tile * kTile + l;
        if (kk >= P.n_act) continue;
        const int64_t r = P.idx ? (int64_t)P.idx[kk] : kk;
        if (r < 0 || r >= P.n) continue;
        if (c < 3) {
            if (P.acc) P.acc[3 * r + c] = P.G * sum;
        } else if (c < 6) {
            if (P.jerk) P.jerk[3 * r + c - 3] = P.G * sum;
        } else if (P.tidal) {
            P.tidal[6 * r + c - 6] = -P.G * sum;
        }
    }
    if (threadIdx.x == 0) P.count[tile] = 0u;   // ready for the next call
}

}  // namespace

// Launch shape: target tiles of 64 and a source split that gives at least
// kDirectBlocks workgroups (so a split happens only with fewer tiles than
// that).  Scratch, with a split: a counter per tile at the start (fixed
// place, zero between calls: the last split of a tile resets it), then one
// FP64 sum per tile, split, component and target.
constexpr int64_t kDirectBlocks = 1024;
constexpr size_t kCountBytes = kDirectBlocks * sizeof(uint32_t);

void ag_direct_shape(int64_t n, int64_t n_act, int64_t* tiles, int64_t* nsplit, int64_t* chunk) {
    const int64_t t = (n_act + kTile - 1) / kTile;
    int64_t s = (kDirectBlocks + t - 1) / t;
    const int64_t max_split = (n + kSrc - 1) / kSrc;
    if (s > max_split) s = max_split;
    if (s > 65535) s = 65535;
    if (s < 1) s = 1;
    int64_t c = (n + s - 1) / s;
    c = (c + kSrc - 1) / kSrc * kSrc;
    *tiles = t;
    *nsplit = (n + c - 1) / c;
    *chunk = c;
}

size_t ag_direct_scratch_bytes(int64_t n, int64_t n_act) {
    int64_t t, s, c;
    ag_direct_shape(n, n_act, &t, &s, &c);
    if (s <= 1) return 0;
    return kCountBytes + (size_t)t * s * kParts * kTile * sizeof(double);
}

size_t ag_direct_count_bytes() { return kCountBytes; }

int ag_launch_direct(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                     const int32_t* idx, int64_t n_act, double eps, double G, int precision,
                     double* acc, double* jerk, double* tidal, void* scratch, bool timed) {
    int64_t tiles, nsplit, chunk;
    ag_direct_shape(n, n_act, &tiles, &nsplit, &chunk);
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
    P.chunk = chunk;
    P.nsplit = (int)nsplit;
    P.count = nsplit > 1 ? reinterpret_cast<uint32_t*>(scratch) : nullptr;
    P.part = nsplit > 1 ? reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) + kCountBytes) : nullptr;
    P.acc = acc;
    P.jerk = jerk;
    P.tidal = tidal;
    P.flags = c->dflags.as<int32_t>();
    PhaseScope phase(c, timed ? AG_PHASE_DIRECT : -1);
    dim3 grid((unsigned)tiles, (unsigned)nsplit);
    hipStream_t st = c->stream;
    const bool fp64 = precision == AG_FP64, per = P.L > 0.0, soft = P.hs != nullptr;
#define AG_DIRECT(A, B, C) hipLaunchKernelGGL((k_direct<A, B, C>), grid, dim3(kThreads), 0, st, P)
    if (fp64) {
        if (per) { if (soft) AG_DIRECT(true, true, true); else AG_DIRECT(true, true, false); }
        else { if (soft) AG_DIRECT(true, false, true); else AG_DIRECT(true, false, false); }
    } else {
        if (per) { if (soft) AG_DIRECT(false, true, true); else AG_DIRECT(false, true, false); }
        else { if (soft) AG_DIRECT(false, false, true); else AG_DIRECT(false, false, false); }
    }
#undef AG_DIRECT
    return AG_OK;
}

// ---------------------------------------------------------------------------
// The allocation-free direct sum, for callers that cannot allocate device
// memory: the split counters and split sums live in a file-scope device array
// of fixed size.  The launch shape bounds the scratch for every size (a split
// happens only with fewer than kDirectBlocks target tiles, so tiles x splits
// < 2 kDirectBlocks), so no call is refused for its size.  Every call on a
// device shares that device's copy of the array: calls that overlap on one
// device race.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocBytes = kCountBytes + (size_t)(2 * kDirectBlocks) * kParts * kTile * sizeof(double);
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
    // the split counters start at zero; each launch leaves them at zero
    e = hipMemset(p, 0, kCountBytes);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return ag_fail(AG_EHIP, "clearing the direct-sum scratch failed: %s", hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return AG_OK;
}

extern "C" int ag_grav_direct_noalloc(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                                      const int32_t* idx, int64_t n_act, double eps, double G, int precision,
                                      double* acc, double* jerk, double* tidal) {
    AG_TRY(ag_direct_check(c, n, x, v, m, idx, n_act, eps, G, precision));
    if (n_act == 0) return AG_OK;
    const size_t bytes = ag_direct_scratch_bytes(n, n_act);
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
