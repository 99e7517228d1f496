// k_tree.hip -- oct-tree construction on the GPU.
//
// Pipeline (all on the context's stream, no host synchronisation):
//   1. bounding cube of each system (order-preserving integer atomics, one
//      atomic per workgroup and axis), non-finite detection;
//   2. 63-bit Morton keys: 21 octal digits; with several systems the top
//      digits hold the system number and the rest its own cube's Morton code;
//   3. stable LSD radix sort of (key, row) pairs over the top 32 key bits,
//      8 bits per pass, then a full-key sort of each level-10 cell that
//      holds more than n_leaf particles;
//   4. x, v, m into key order (FP64 and FP32 copies);
//   5. topology straight from the sorted keys: with c_p the number of octal
//      digits key[p] shares with key[p-1], the cell of level l that contains
//      position p starts at p iff c_p < l.  A cell is split while it holds
//      more than n_leaf particles (and below level 21); system-prefix levels
//      are always split.  Counting, per position, the cells that start there
//      and exist in the tree, then an exclusive scan, numbers the nodes in
//      depth-first pre-order: node (l, p) has id off[p] + l - c_p - 1, its
//      first child is id + 1 and its "skip" link (next node outside its
//      subtree) is off[e], e = the first position past the cell;
//   6. moments level by level from the deepest, in FP64: leaves from their
//      particles, inner nodes from their children, each in one pass about
//      its first member, shifted to the centre of mass at the end.
#include <float.h>

#include <algorithm>
#include <climits>

#include "ag_internal.h"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float f_down(double d) {
    float f = (float)d;
    if ((double)f > d) f = nextafterf(f, -FLT_MAX);
    return f;
}
__device__ __forceinline__ float f_up(double d) {
    float f = (float)d;
    if ((double)f < d) f = nextafterf(f, FLT_MAX);
    return f;
}

__device__ __forceinline__ int sys_of(const int64_t* __restrict__ off, int n_sys, int64_t i) {
    int lo = 0, hi = n_sys;   // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// 1. bounding cubes
// ---------------------------------------------------------------------------
constexpr int64_t kBoxChunk = 2048;

// One block opens a build: system offsets (checked; NULL = one system), the
// empty bounding boxes, the first box workgroup of each system (exclusive
// scan of their chunk counts) and a zeroed tree header.
__global__ void k_build_init(int n_sys, int64_t n, const int64_t* __restrict__ in, int64_t* __restrict__ off,
                             int32_t* __restrict__ flags, uint64_t* __restrict__ box, int32_t* __restrict__ blk_off,
                             int64_t* __restrict__ hdr, int hdr_words) {
    __shared__ int s_sum[AG_MAX_SYS + 1];
    for (int s = threadIdx.x; s <= n_sys; s += blockDim.x) {
        const int64_t v = in ? in[s] : (s == 0 ? 0 : n);
        if (in) {
            const bool bad = (s == 0 && v != 0) || (s == n_sys && v != n) || v < 0 || v > n ||
                             (s > 0 && in[s - 1] > v);
            if (bad) atomicOr(flags, AGF_BADINDEX);
        }
        off[s] = v;
    }
    for (int i = threadIdx.x; i < hdr_words; i += blockDim.x) hdr[i] = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < n_sys; s += blockDim.x) {
        for (int c = 0; c < 3; ++c) {
            box[6 * s + c] = ~0ull;        // min slots start at the top
            box[6 * s + 3 + c] = 0ull;     // max slots at the bottom
        }
        const int64_t sz = off[s + 1] - off[s];
        s_sum[s] = (int)((sz + kBoxChunk - 1) / kBoxChunk);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int s = 0; s < n_sys; ++s) {
            const int v = s_sum[s];
            blk_off[s] = acc;
            acc += v;
        }
        blk_off[n_sys] = acc;
    }
}

// A periodic tree holds every position in the primary cube [0, pbox): the
// image is immaterial to the forces, and compact cells keep groups compact.
__device__ __forceinline__ double in_box(double q, double pbox) {
    return pbox > 0.0 ? q - pbox * floor(q / pbox) : q;
}

// Each workgroup of 384 threads (a multiple of 3, so a thread always meets
// the same coordinate) reads kBoxChunk consecutive rows as one contiguous run
// of doubles and writes its per-coordinate minima and maxima (order-preserving
// integers) to part[6 b ..]; k_box_reduce combines the workgroups of each
// system.  Non-finite coordinates raise the flag and are left out.
constexpr int kBoxThreads = 384;

__global__ void __launch_bounds__(kBoxThreads) k_box(const double* __restrict__ x, const int64_t* __restrict__ off,
                                                     int n_sys, const int32_t* __restrict__ blk_off,
                                                     uint64_t* __restrict__ part, int32_t* __restrict__ flags,
                                                     double pbox) {
    __shared__ uint64_t s_red[6][kBoxThreads / 64];
    const int b = blockIdx.x;
    if (b >= blk_off[n_sys]) return;
    int lo = 0, hi = n_sys;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (blk_off[mid] <= b) lo = mid; else hi = mid;
    }
    const int s = lo;
    const int64_t i0 = off[s] + (int64_t)(b - blk_off[s]) * kBoxChunk;
    const int64_t i1 = i0 + kBoxChunk < off[s + 1] ? i0 + kBoxChunk : off[s + 1];
    const int c = threadIdx.x % 3;   // kBoxThreads is a multiple of 3
    double mn = DBL_MAX, mx = -DBL_MAX;
    bool bad = false;
    // all of the thread's loads issued before any is used
    constexpr int kPer = 3 * kBoxChunk / kBoxThreads;
    double q[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t j = 3 * i0 + threadIdx.x + (int64_t)k * kBoxThreads;
        q[k] = j < 3 * i1 ? x[j] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (3 * i0 + threadIdx.x + (int64_t)k * kBoxThreads >= 3 * i1) continue;
        if (!isfinite(q[k])) {
            bad = true;
            continue;
        }
        const double u = in_box(q[k], pbox);
        mn = u < mn ? u : mn;
        mx = u > mx ? u : mx;
    }
    if (bad) atomicOr(flags, AGF_NONFINITE);
    // per coordinate: the wave's lanes of that coordinate, then the waves
    uint64_t omn[3], omx[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        omn[k] = ag_wave_min(k == c ? ag_ord(mn) : ~0ull);
        omx[k] = ag_wave_max(k == c ? ag_ord(mx) : 0ull);
    }
    const int lane = ag_lane(), w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_red[k][w] = omn[k];
            s_red[3 + k][w] = omx[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        uint64_t r = s_red[k][0];
        for (int q = 1; q < kBoxThreads / 64; ++q) r = k < 3 ? (s_red[k][q] < r ? s_red[k][q] : r)
                                                           : (s_red[k][q] > r ? s_red[k][q] : r);
        part[6 * (int64_t)b + k] = r;
    }
}

// one workgroup per system: its box from the partial boxes of its workgroups
__global__ void k_box_reduce(int n_sys, const int32_t* __restrict__ blk_off, const uint64_t* __restrict__ part,
                             uint64_t* __restrict__ box) {
    __shared__ uint64_t s_red[6][4];
    const int s = blockIdx.x;
    if (s >= n_sys) return;
    uint64_t v[6] = {~0ull, ~0ull, ~0ull, 0ull, 0ull, 0ull};
    for (int b = blk_off[s] + threadIdx.x; b < blk_off[s + 1]; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const uint64_t q = part[6 * (int64_t)b + k];
            v[k] = k < 3 ? (q < v[k] ? q : v[k]) : (q > v[k] ? q : v[k]);
        }
    const int lane = ag_lane(), w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const uint64_t r = k < 3 ? ag_wave_min(v[k]) : ag_wave_max(v[k]);
        if (lane == 0) s_red[k][w] = r;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        uint64_t r = s_red[k][0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r = k < 3 ? (s_red[k][q] < r ? s_red[k][q] : r)
                                                                  : (s_red[k][q] > r ? s_red[k][q] : r);
        box[6 * s + k] = r;
    }
}

// ---------------------------------------------------------------------------
// 2. Morton keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    // spread the low 21 bits of v to every third bit
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__global__ void k_keys(int64_t n, const double* __restrict__ x, const int64_t* __restrict__ off, int n_sys,
                       int bits, const uint64_t* __restrict__ box, uint64_t* __restrict__ keys,
                       int32_t* __restrict__ vals, double pbox) {
    const double scale_cells = (double)(1u << bits);
    const int64_t maxc = ((int64_t)1 << bits) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int s = n_sys > 1 ? sys_of(off, n_sys, i) : 0;
        double lo[3], ext = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = ag_unord(box[6 * s + c]);
            double e = ag_unord(box[6 * s + 3 + c]) - lo[c];
            ext = e > ext ? e : ext;
        }
        if (!(ext > 0.0) || !isfinite(ext)) ext = 1.0;
        if (pbox > 0.0) {   // a periodic tree's root cell is the box itself
            lo[0] = lo[1] = lo[2] = 0.0;
            ext = pbox;
        }
        // (a periodic root is split exactly at half the box: no cell below it
        // crosses the planes where sources change image about a multiple of
        // half the box)
        const double inv = pbox > 0.0 ? scale_cells / pbox : scale_cells / (ext * (1.0 + 1e-12));
        uint64_t code = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double q = (in_box(x[3 * i + c], pbox) - lo[c]) * inv;
            int64_t k = isfinite(q) ? (int64_t)q : 0;
            k = k < 0 ? 0 : (k > maxc ? maxc : k);
            code |= spread3((uint64_t)k) << (2 - c);
        }
        keys[i] = ((uint64_t)s << (3 * bits)) | code;
        vals[i] = (int32_t)i;
    }
}

// ---------------------------------------------------------------------------
// 3. stable LSD radix sort, 8 bits per pass
// ---------------------------------------------------------------------------
constexpr int kRsItems = 16;
constexpr int kRsTile = kThreads * kRsItems;

__global__ void __launch_bounds__(kThreads) k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                      int nblocks, int32_t* __restrict__ hist) {
    __shared__ int s_h[4][256];
    for (int w = 0; w < 4; ++w) s_h[w][threadIdx.x] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        int64_t i = base + k * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&s_h[w][(keys[i] >> shift) & 255], 1);
    }
    __syncthreads();
    int t = s_h[0][threadIdx.x] + s_h[1][threadIdx.x] + s_h[2][threadIdx.x] + s_h[3][threadIdx.x];
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = t;
}

// exclusive scan of one value per thread over a 256-thread block; *total
// receives the block's sum
__device__ __forceinline__ int block_excl_scan256(int v, int* s_tmp, int* total) {
    const int lane = ag_lane(), w = threadIdx.x >> 6;
    const int inc = ag_wave_incl_scan(v);
    if (lane == 63) s_tmp[w] = inc;
    __syncthreads();
    int pre = 0, all = 0;
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) {
        pre += q < w ? s_tmp[q] : 0;
        all += s_tmp[q];
    }
    __syncthreads();
    *total = all;
    return pre + inc - v;
}

// Per digit d (one block each): exclusive scan of the per-block counts
// hist[d][0 .. nblocks) into hoff, and the digit's total into tot[d].
__global__ void __launch_bounds__(kThreads) k_rs_rowscan(const int32_t* __restrict__ hist, int nblocks,
                                                         int32_t* __restrict__ hoff, int32_t* __restrict__ tot) {
    __shared__ int s_tmp[kThreads / 64];
    const int64_t row = (int64_t)blockIdx.x * nblocks;
    int carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += kThreads) {
        const int b = b0 + threadIdx.x;
        const int v = b < nblocks ? hist[row + b] : 0;
        int sum;
        const int ex = block_excl_scan256(v, s_tmp, &sum);
        if (b < nblocks) hoff[row + b] = carry + ex;
        carry += sum;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Stable scatter of one tile of (key, value) pairs by one 8-bit digit.  Each
// wave ranks its own contiguous run of the tile (kRsItems rows of 64) with no
// workgroup barrier: lanes with equal digits are matched by ballots, and the
// wave keeps a running count per digit in its own LDS row, read by all the
// matched lanes before their first lane adds the group's size.  One scan per
// digit over the four waves then places every element in the tile's
// digit-ordered LDS copy, which is written out so that each digit's run goes
// to consecutive addresses.  With `rank` set (last pass), rank[value]
// receives the value's final position.
__global__ void __launch_bounds__(kThreads) k_rs_scatter(const uint64_t* __restrict__ kin,
                                                         const int32_t* __restrict__ vin, int64_t n,
                                                         int shift, int nblocks,
                                                         const int32_t* __restrict__ hist,
                                                         const int32_t* __restrict__ hoff,
                                                         const int32_t* __restrict__ tot,
                                                         uint64_t* __restrict__ kout,
                                                         int32_t* __restrict__ vout,
                                                         int32_t* __restrict__ rank) {
    __shared__ uint64_t s_key[kRsTile];
    __shared__ int s_val[kRsTile];
    __shared__ int s_gofs[256];   // global position of the tile's first digit-d element minus its tile slot
    __shared__ int s_loc[256];    // tile slot of the first digit-d element
    __shared__ int s_w[4][256];   // per-wave digit counts, then per-wave offsets within the digit
    __shared__ int s_tmp[kThreads / 64];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    {
        int all;
        const int base_d = block_excl_scan256(tot[t], s_tmp, &all);
        const int loc = block_excl_scan256(hist[(int64_t)t * nblocks + blockIdx.x], s_tmp, &all);
        s_loc[t] = loc;
        s_gofs[t] = base_d + hoff[(int64_t)t * nblocks + blockIdx.x] - loc;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s_w[q][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)w * (kRsItems * 64);
    uint64_t key[kRsItems];
    int32_t val[kRsItems];
    int rk[kRsItems];
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t i = base + k * 64 + lane;
        const bool valid = i < n;
        key[k] = valid ? kin[i] : 0ull;
        val[k] = valid ? vin[i] : 0;
    }
    int* cnt_w = s_w[w];
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        const bool valid = base + k * 64 + lane < n;
        const int d = (int)((key[k] >> shift) & 255);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const int r = ag_prefix_count(peers);
        int before = 0;
        if (valid) before = cnt_w[d];   // every matched lane reads the count ...
        if (valid && r == 0) cnt_w[d] = before + __popcll(peers);   // ... before the first one adds to it
        rk[k] = before + r;
    }
    __syncthreads();
    {
        int run = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = s_w[q][t];
            s_w[q][t] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRsItems; ++k) {
        if (base + k * 64 + lane < n) {
            const int d = (int)((key[k] >> shift) & 255);
            const int slot = s_loc[d] + cnt_w[d] + rk[k];
            s_key[slot] = key[k];
            s_val[slot] = val[k];
        }
    }
    __syncthreads();
    const int64_t rem = n - (int64_t)blockIdx.x * kRsTile;
    const int nvalid = rem < kRsTile ? (int)rem : kRsTile;
    for (int j = t; j < nvalid; j += kThreads) {
        const uint64_t kj = s_key[j];
        const int d = (int)((kj >> shift) & 255);
        const int pos = s_gofs[d] + j;
        kout[pos] = kj;
        const int32_t vj = s_val[j];
        vout[pos] = vj;
        if (rank) rank[vj] = pos;
    }
}

int grid_for(int64_t n, int threads = kThreads) {
    int64_t b = (n + threads - 1) / threads;
    if (b > 8192) b = 8192;
    return (int)(b < 1 ? 1 : b);
}

// ---------------------------------------------------------------------------
// 4. particle data into key order: coalesced reads in input order, each row
//    written to its sorted position (scattered 32-byte stores, which the
//    last-level cache merges before they reach HBM).  Velocities are not
//    written in key order: the leaf moments read them through the sorted
//    rows (perm) and write the FP32 copies the walk uses, in order.
//    (Reading the positions that way too, with no scatter at all, was slower
//    on randomly ordered input: the gathered 24-byte reads cost more than
//    the merged stores.)
// ---------------------------------------------------------------------------
__global__ void k_to_sorted_pos(int64_t n, const int32_t* __restrict__ rank, const double* __restrict__ x,
                                const double* __restrict__ m, double4* __restrict__ spos, double pbox,
                                const double* __restrict__ h, float* __restrict__ sh) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = rank[i];
        spos[p] = make_double4(in_box(x[3 * i], pbox), in_box(x[3 * i + 1], pbox), in_box(x[3 * i + 2], pbox), m[i]);
        if (h) sh[p] = f_up(h[i]);   // per-particle softening, rounded up
    }
}
void launch_to_sorted(ag_ctx* c, int64_t n, const double* x, const double* m, double pbox) {
    const int32_t* rank = c->rank.as<int32_t>();
    hipLaunchKernelGGL(k_to_sorted_pos, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, n, rank, x, m,
                       c->spos.as<double4>(), pbox, c->tree_soft ? c->soft_h.as<double>() : nullptr,
                       c->soft_s.as<float>());
}

// ---------------------------------------------------------------------------
// 5. topology
// ---------------------------------------------------------------------------
__device__ __forceinline__ int common_digits(uint64_t a, uint64_t b) {
    const uint64_t d = a ^ b;
    if (d == 0) return AG_MAX_LEVEL;
    return (__clzll(d) - 1) / 3;   // bit 63 is always clear
}

// Minima of the shared-digit counts over aligned runs of 16^(k+1) positions,
// k = 0 .. 5 (16 positions up to 2^24): the search for a far cell end skips
// whole runs with them.  Levels 0-2 are written by k_cdig (a workgroup pass
// covers 4096 positions), levels 3-5 by k_cd_min_top.
constexpr int kCdLevels = 6;
struct CdMin {
    int32_t* lev[kCdLevels];
};
constexpr int kRun = 256;                 // threads of k_cdig
constexpr int64_t kCdPass = 16 * kRun;   // positions per k_cdig workgroup pass

__global__ void __launch_bounds__(kRun) k_cdig(int64_t n, const uint64_t* __restrict__ keys, int32_t* __restrict__ cd,
                                               CdMin M) {
    __shared__ int s_w[16][kRun / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t g = blockIdx.x; g * kCdPass < n; g += gridDim.x) {
        for (int j = 0; j < 16; ++j) {
            const int64_t p = g * kCdPass + j * kRun + threadIdx.x;
            int v = INT_MAX;
            if (p < n) {
                v = p == 0 ? -1 : common_digits(keys[p - 1], keys[p]);
                cd[p] = v;
            }
            int m16 = v;   // runs of 16 (level 0)
            m16 = min(m16, __shfl_xor(m16, 1, 16));
            m16 = min(m16, __shfl_xor(m16, 2, 16));
            m16 = min(m16, __shfl_xor(m16, 4, 16));
            m16 = min(m16, __shfl_xor(m16, 8, 16));
            if ((threadIdx.x & 15) == 0) M.lev[0][p >> 4] = m16;
            const int wv = ag_wave_min(v);
            if (lane == 0) s_w[j][w] = wv;
        }
        __syncthreads();
        if (threadIdx.x < 16) {   // runs of 256 (level 1), then of 4096 (level 2)
            int m = s_w[threadIdx.x][0];
            for (int k = 1; k < kRun / 64; ++k) m = s_w[threadIdx.x][k] < m ? s_w[threadIdx.x][k] : m;
            M.lev[1][g * 16 + threadIdx.x] = m;
            m = min(m, __shfl_xor(m, 1, 16));
            m = min(m, __shfl_xor(m, 2, 16));
            m = min(m, __shfl_xor(m, 4, 16));
            m = min(m, __shfl_xor(m, 8, 16));
            if (threadIdx.x == 0) M.lev[2][g] = m;
        }
        __syncthreads();
    }
}

// levels 3-5 from level 2 (one workgroup); cnt[k] entries at level k
struct CdCounts {
    int64_t cnt[kCdLevels];
};
__global__ void k_cd_min_top(CdMin M, CdCounts C) {
    for (int k = 3; k < kCdLevels; ++k) {
        for (int64_t i = threadIdx.x; i < C.cnt[k]; i += blockDim.x) {
            int m = INT_MAX;
            for (int j = 0; j < 16; ++j) {
                const int64_t q = 16 * i + j;
                if (q < C.cnt[k - 1]) m = min(m, M.lev[k - 1][q]);
            }
            M.lev[k][i] = m;
        }
        __syncthreads();
    }
}

// first position q' >= q with cd[q'] < l (n if none): finish q's run of 16,
// then skip whole runs by their minima, climbing a level each time a run of
// the level above is passed, and search the run found downwards
__device__ int64_t next_below(int64_t n, const int32_t* __restrict__ cd, const CdMin& M, int64_t q, int l) {
    if (q >= n) return n;
    for (; q & 15; ++q) {
        if (q >= n) return n;
        if (cd[q] < l) return q;
    }
    int lev = 0;
    int64_t idx = q >> 4;
    for (;;) {
        if ((idx << (4 * (lev + 1))) >= n) return n;
        if (M.lev[lev][idx] < l) break;
        ++idx;
        if ((idx & 15) == 0 && lev < kCdLevels - 1) {
            ++lev;
            idx >>= 4;
        }
    }
    while (lev > 0) {
        --lev;
        idx <<= 4;
        while (M.lev[lev][idx] >= l) ++idx;
    }
    q = idx << 4;
    while (cd[q] >= l) ++q;
    return q;
}

struct TopoParams {
    int64_t n;
    int n_leaf;
    int sys_levels;
};

// Nodes starting at each position, and how many of them are inner nodes
// (all but the last, which is a leaf), from a window of the shared-digit
// counts in LDS (cd' = -1 past the end, so the end bounds every cell):
//  - the node at level c + 1 (c = cd[p]) exists iff p = 0 or the level-c cell
//    holding p is split: c below the system levels, or c < 21 and the cell
//    (from the last a < p with cd[a] < c to the first q > p with cd'[q] < c)
//    holds more than n_leaf particles;
//  - the cell of level l starting at p holds at most n_leaf particles iff
//    some q in (p, p + n_leaf] has cd'[q] < l, i.e. iff l > mn, mn the
//    minimum of cd' there; so the leaf is at L = max(c + 1, system levels,
//    min(21, mn + 1)) and L - c nodes start at p.
constexpr int kWin = 64;   // largest n_leaf

__global__ void __launch_bounds__(kThreads) k_count_nodes(TopoParams P, const int32_t* __restrict__ cd,
                                                          int32_t* __restrict__ cnt, int32_t* __restrict__ icnt) {
    __shared__ int s_cd[kThreads + 2 * kWin];
    const int W = P.n_leaf;
    for (int64_t p0 = (int64_t)blockIdx.x * kThreads; p0 < P.n; p0 += (int64_t)gridDim.x * kThreads) {
        __syncthreads();
        for (int k = threadIdx.x; k < kThreads + 2 * W; k += kThreads) {
            const int64_t q = p0 - W + k;
            s_cd[k] = (q >= 0 && q < P.n) ? cd[q] : -1;
        }
        __syncthreads();
        const int64_t p = p0 + threadIdx.x;
        if (p >= P.n) continue;
        const int* w = s_cd + W + threadIdx.x;   // w[0] = cd[p], w[k] = cd'[p + k]
        const int c = w[0];
        int k = 0;
        bool exists = true;
        if (p > 0) {
            if (c >= AG_MAX_LEVEL) {
                exists = false;
            } else if (c >= P.sys_levels) {
                int db = 0, df = 0;   // distance back to the cell's start, forward to its end (0: beyond the window)
                for (int j = 1; j <= W; ++j)
                    if (!db && p - j >= 0 && w[-j] < c) db = j;
                for (int j = 1; j <= W; ++j)
                    if (!df && w[j] < c) df = j;
                exists = !db || !df || db + df > W;
            }
        }
        if (exists) {
            int mn = INT_MAX;
            for (int j = 1; j <= W; ++j) mn = w[j] < mn ? w[j] : mn;
            int L = mn + 1 < AG_MAX_LEVEL ? mn + 1 : AG_MAX_LEVEL;
            L = L > c + 1 ? L : c + 1;
            L = L > P.sys_levels ? L : P.sys_levels;
            k = L - c;
        }
        cnt[p] = k;
        icnt[p] = k > 0 ? k - 1 : 0;
    }
}

// first position after p whose key differs from key[p] in the top l digits
// (galloping search: cells are usually short compared with n)
__device__ __forceinline__ int64_t cell_end(const TopoParams& P, const uint64_t* __restrict__ keys, int64_t p,
                                            int l) {
    if (l == 0) return P.n;
    const int sh = 63 - 3 * l;
    const uint64_t pre = keys[p] >> sh;
    int64_t lo = p + 1, step = 16, hi = P.n;
    while (lo + step < P.n) {
        if ((keys[lo + step] >> sh) != pre) {
            hi = lo + step;
            break;
        }
        lo += step + 1;
        step <<= 1;
    }
    while (lo < hi) {   // answer in [lo, hi]
        const int64_t mid = (lo + hi) >> 1;
        if ((keys[mid] >> sh) == pre) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// ---- dense cells (the last step of the sort, which needs cell_end) ----
// The passes order the keys by bits 31..62 only: every level-10 cell (bits
// 33..62) ends up contiguous, and the tree splits no cell below level 10
// unless it holds more than n_leaf particles.  Those cells alone are then
// sorted by their full keys (rows break ties, which is the order a stable
// sort of the full keys gives); the order inside the other level-10 cells
// is never looked at below their leaf level.
constexpr int kSortedShift = 31;
constexpr int kCellShift = 33;
constexpr int kSegLds = 2048;   // cells up to this size sort in LDS

__global__ void k_seg_heads(int64_t n, const uint64_t* __restrict__ k, int n_leaf, int32_t* __restrict__ flag) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t c = k[p] >> kCellShift;
        const bool head = p == 0 || (k[p - 1] >> kCellShift) != c;
        flag[p] = head && p + n_leaf < n && (k[p + n_leaf] >> kCellShift) == c;
    }
}

__global__ void k_seg_list(int64_t n, const int32_t* __restrict__ flag, const int32_t* __restrict__ off,
                           int32_t* __restrict__ list) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        if (flag[p]) list[off[p]] = (int32_t)p;
}

__device__ __forceinline__ bool pair_greater(uint64_t ka, int va, uint64_t kb, int vb) {
    return ka > kb || (ka == kb && va > vb);
}

// One workgroup per dense cell [a, e): bitonic sort in LDS up to kSegLds
// entries, else a stable LSD radix sort of bits 0..34 (5 passes of 7 bits)
// through the spare key buffers at the same positions.
__global__ void __launch_bounds__(kThreads) k_seg_sort(TopoParams P, const int32_t* __restrict__ list,
                                                       const int32_t* __restrict__ count, uint64_t* __restrict__ k0,
                                                       int32_t* __restrict__ perm, int32_t* __restrict__ rank,
                                                       uint64_t* __restrict__ k1, int32_t* __restrict__ v1) {
    __shared__ uint64_t s_k[kSegLds];
    __shared__ int32_t s_v[kSegLds];
    __shared__ int s_base[128];
    __shared__ int s_w[kThreads / 64][128];
    const int tid = threadIdx.x;
    const int ns = *count;
    for (int s = blockIdx.x; s < ns; s += gridDim.x) {
        const int64_t a = list[s];
        const int64_t L = cell_end(P, k0, a, 10) - a;
        if (L <= kSegLds) {
            int Pw = 1;
            while (Pw < L) Pw <<= 1;
            for (int i = tid; i < Pw; i += kThreads) {
                s_k[i] = i < L ? k0[a + i] : ~0ull;    // real keys have bit 63 clear
                s_v[i] = i < L ? perm[a + i] : 0x7fffffff;
            }
            __syncthreads();
            for (int kk = 2; kk <= Pw; kk <<= 1)
                for (int j = kk >> 1; j > 0; j >>= 1) {
                    for (int i = tid; i < Pw; i += kThreads) {
                        const int ixj = i ^ j;
                        if (ixj > i) {
                            const bool up = (i & kk) == 0;
                            if (pair_greater(s_k[i], s_v[i], s_k[ixj], s_v[ixj]) == up) {
                                const uint64_t tk = s_k[i];
                                s_k[i] = s_k[ixj];
                                s_k[ixj] = tk;
                                const int32_t tv = s_v[i];
                                s_v[i] = s_v[ixj];
                                s_v[ixj] = tv;
                            }
                        }
                    }
                    __syncthreads();
                }
            for (int i = tid; i < L; i += kThreads) {
                k0[a + i] = s_k[i];
                perm[a + i] = s_v[i];
                rank[s_v[i]] = (int32_t)(a + i);
            }
            __syncthreads();
            continue;
        }
        const int w = tid >> 6;
        for (int pass = 0; pass < 5; ++pass) {
            const int shift = 7 * pass;
            const uint64_t* ks = (pass & 1) ? k1 : k0;
            const int32_t* vs = (pass & 1) ? v1 : perm;
            uint64_t* kd = (pass & 1) ? k0 : k1;
            int32_t* vd = (pass & 1) ? perm : v1;
            if (tid < 128) s_base[tid] = 0;
            __syncthreads();
            for (int64_t i = tid; i < L; i += kThreads) atomicAdd(&s_base[(int)((ks[a + i] >> shift) & 127)], 1);
            __syncthreads();
            if (tid == 0) {
                int acc = 0;
                for (int d = 0; d < 128; ++d) {
                    const int c = s_base[d];
                    s_base[d] = acc;
                    acc += c;
                }
            }
            __syncthreads();
            for (int64_t c0 = 0; c0 < L; c0 += kThreads) {
                const int64_t i = c0 + tid;
                const bool valid = i < L;
                const uint64_t key = valid ? ks[a + i] : 0ull;
                const int32_t val = valid ? vs[a + i] : 0;
                const int d = (int)((key >> shift) & 127);
                uint64_t peers = __ballot(valid);
#pragma unroll
                for (int b = 0; b < 7; ++b) {
                    const bool bit = (d >> b) & 1;
                    const uint64_t bb = __ballot(bit);
                    peers &= bit ? bb : ~bb;
                }
                const int r = ag_prefix_count(peers);
                const int cnt = __popcll(peers);
                if (tid < 128)
                    for (int q = 0; q < kThreads / 64; ++q) s_w[q][tid] = 0;
                __syncthreads();
                if (valid && r == 0) s_w[w][d] = cnt;
                __syncthreads();
                if (tid < 128) {
                    int run = s_base[tid];
                    for (int q = 0; q < kThreads / 64; ++q) {
                        const int c = s_w[q][tid];
                        s_w[q][tid] = run;
                        run += c;
                    }
                    s_base[tid] = run;
                }
                __syncthreads();
                if (valid) {
                    const int64_t pos = a + s_w[w][d] + r;
                    kd[pos] = key;
                    vd[pos] = val;
                }
                __syncthreads();
            }
        }
        // five passes end in the spare buffers: copy back
        for (int64_t i = tid; i < L; i += kThreads) {
            k0[a + i] = k1[a + i];
            const int32_t v = v1[a + i];
            perm[a + i] = v;
            rank[v] = (int32_t)(a + i);
        }
        __syncthreads();
    }
}

// Writes every node's link and lists the inner nodes (in pre-order) and the
// leaves with their first positions.  The end of the cell of node (l, p) is
// the first q > p with cd'[q] < l; ends do not decrease from the deepest node
// at p (the leaf) to the shallowest, so each search continues from the end
// below it.  Every wave works on its own run of 64 positions with its own LDS
// window (the run and kWaveLook positions past it: the shared-digit counts,
// their minima per 16 and the node offsets, so a skip inside the window
// costs no global load), and no wave waits at a workgroup barrier for
// another's searches.  A node whose
// end lies beyond the window, and every node above it at p, is left to
// k_far_ends: p and the deepest such node go to a list (their skip and count
// fields are written there), gathered per wave in LDS and appended to the
// global list with one atomic per workgroup (or per wave when its LDS list
// fills).  The inner nodes per level and the deepest level go to
// per-workgroup slots that k_tree_close adds up.
constexpr int kWriteBlocks = 2048;   // eight workgroups per CU at most
constexpr int kWaveLook = 208;       // positions searched past a wave's run (>= n_leaf + 1)
constexpr int kWaveWin = 64 + kWaveLook;   // 17 runs of 16
constexpr int kWinRuns = kWaveWin / 16;
constexpr int kFarWave = 256;        // far entries held per wave between flushes
constexpr int kLevels = AG_MAX_LEVEL + 1;

// orders a wave's LDS accesses around it (the wave's lanes share the window)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// index of the first entry at or after j in one run of 16 window entries
// (four 16-byte reads) that is below l, or INT_MAX
__device__ __forceinline__ int run_first_below(const int* __restrict__ cdw, int run, int j, int l) {
    int r = INT_MAX;
#pragma unroll
    for (int g = 3; g >= 0; --g) {   // from the back: the first hit wins
        const int4 v = reinterpret_cast<const int4*>(cdw)[4 * run + g];
        const int b = 16 * run + 4 * g;
        r = (b + 3 >= j && v.w < l) ? b + 3 : r;
        r = (b + 2 >= j && v.z < l) ? b + 2 : r;
        r = (b + 1 >= j && v.y < l) ? b + 1 : r;
        r = (b >= j && v.x < l) ? b : r;
    }
    return r;
}

// First window index q >= j with a shared-digit count below l, or kWaveWin
// if none: the run holding j, then the first later run whose minimum is
// below l (all kWinRuns minima read at once), then that run.  Fixed-length
// reads instead of a scan that stops at the hit keep the scalar unit, which
// the divergent loops of a scan keep busy, free.
__device__ __forceinline__ int win_first_below(const int* __restrict__ cdw, const int* __restrict__ m16w, int j,
                                               int l) {
    if (j >= kWaveWin) return kWaveWin;
    const int rj = j >> 4;
    int q = run_first_below(cdw, rj, j, l);
    if (q != INT_MAX) return q;
    int rf = INT_MAX;
#pragma unroll
    for (int g = (kWinRuns + 3) / 4 - 1; g >= 0; --g) {
        const int4 m = reinterpret_cast<const int4*>(m16w)[g];
        rf = (4 * g + 3 > rj && 4 * g + 3 < kWinRuns && m.w < l) ? 4 * g + 3 : rf;
        rf = (4 * g + 2 > rj && 4 * g + 2 < kWinRuns && m.z < l) ? 4 * g + 2 : rf;
        rf = (4 * g + 1 > rj && 4 * g + 1 < kWinRuns && m.y < l) ? 4 * g + 1 : rf;
        rf = (4 * g > rj && m.x < l) ? 4 * g : rf;
    }
    if (rf == INT_MAX) return kWaveWin;
    return run_first_below(cdw, rf, 0, l);
}

__global__ void __launch_bounds__(kThreads) k_write_nodes(TopoParams P, const int32_t* __restrict__ cd,
                                                          const int32_t* __restrict__ off,
                                                          const int32_t* __restrict__ ioff, int4* __restrict__ link,
                                                          int32_t* __restrict__ ilist, int32_t* __restrict__ leaves,
                                                          int32_t* __restrict__ leaf_pos,
                                                          int64_t* __restrict__ hdr, int32_t* __restrict__ blk,
                                                          int32_t* __restrict__ far_p, int32_t* __restrict__ far_t) {
    constexpr int kWaves = kThreads / 64;
    __shared__ int s_lc[kLevels];   // inner nodes of this workgroup per level
    __shared__ __align__(16) int s_cd[kWaves][kWaveWin];
    __shared__ int s_off[kWaves][kWaveWin];
    __shared__ __align__(16) int s_m16[kWaves][(kWinRuns + 3) / 4 * 4];
    __shared__ int s_fp[kWaves][kFarWave], s_ft[kWaves][kFarWave];
    __shared__ int s_fn[kWaves], s_fbase;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x < kLevels) s_lc[threadIdx.x] = 0;
    if (lane == 0) s_fn[w] = 0;
    __syncthreads();
    int* cdw = s_cd[w];
    int* offw = s_off[w];
    int* m16w = s_m16[w];
    constexpr int LW = kWaveWin;
    const int64_t n_nodes = off[P.n];
    int maxl = 0;
    for (int64_t p0 = ((int64_t)blockIdx.x * kWaves + w) * 64; p0 < P.n; p0 += (int64_t)gridDim.x * kThreads) {
        wave_sync();
        const int nf = s_fn[w];
        if (nf > kFarWave - 64) {   // room for this run's entries: flush the wave's list
            int base = 0;
            if (lane == 0) base = atomicAdd(reinterpret_cast<int32_t*>(hdr + 3), nf);
            base = __shfl(base, 0, 64);
            for (int i = lane; i < nf; i += 64) {
                far_p[base + i] = s_fp[w][i];
                far_t[base + i] = s_ft[w][i];
            }
            wave_sync();
            if (lane == 0) s_fn[w] = 0;
        }
        for (int k = lane; k < LW; k += 64) {
            const int64_t q = p0 + k;
            cdw[k] = q < P.n ? cd[q] : -1;   // -1 past the end: it ends every cell
            offw[k] = q <= P.n ? off[q] : 0;
        }
        wave_sync();
        if (lane < kWinRuns) {
            int m = cdw[16 * lane];
            for (int j = 1; j < 16; ++j) m = min(m, cdw[16 * lane + j]);
            m16w[lane] = m;
        }
        wave_sync();
        const int64_t p = p0 + lane;
        if (p >= P.n) continue;
        const int op = offw[lane];
        const int k = offw[lane + 1] - op;
        if (k == 0) continue;
        const int iop = ioff[p];
        const int c = cdw[lane];
        int j = lane + 1;   // search position (window index)
        bool far = false;
        for (int t = k - 1; t >= 0; --t) {
            const int l = c + 1 + t;
            int64_t e = -1;
            if (!far) {
                j = win_first_below(cdw, m16w, j, l);
                if (j < LW) e = p0 + j;
                if (e < 0) {   // beyond the window: this node and the ones above it
                    far = true;
                    const int q = atomicAdd(&s_fn[w], 1);
                    s_fp[w][q] = (int)p;
                    s_ft[w][q] = t;
                }
            }
            const bool leaf = (t == k - 1);
            const int64_t id = op + t;
            const int skip = far ? 0 : offw[e - p0];   // off[n] = n_nodes past the end
            link[id] = make_int4(skip, (int)p, far ? 0 : (int)(e - p), l | (leaf ? 0x100 : 0));
            if (!leaf) {
                ilist[iop + t] = (int32_t)id;
                atomicAdd(&s_lc[l], 1);
            } else {
                const int64_t lf = op - iop;   // leaves before p = nodes - inner nodes before p
                leaves[lf] = (int32_t)id;
                leaf_pos[lf] = (int32_t)p;
            }
            maxl = l > maxl ? l : maxl;
        }
    }
    // the workgroup's far entries: one global atomic for all its waves
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int q = 0; q < kWaves; ++q) tot += s_fn[q];
        s_fbase = tot ? atomicAdd(reinterpret_cast<int32_t*>(hdr + 3), tot) : 0;
    }
    __syncthreads();
    {
        int base = s_fbase;
        for (int q = 0; q < w; ++q) base += s_fn[q];
        for (int i = lane; i < s_fn[w]; i += 64) {
            far_p[base + i] = s_fp[w][i];
            far_t[base + i] = s_ft[w][i];
        }
    }
    // per-workgroup inner nodes per level and deepest level, reduced by k_tree_close
    __shared__ int s_max[kWaves];
    maxl = ag_wave_max(maxl);
    if (lane == 0) s_max[w] = maxl;
    __syncthreads();
    int32_t* row = blk + (int64_t)blockIdx.x * (kLevels + 1);
    if (threadIdx.x < kLevels) row[threadIdx.x] = s_lc[threadIdx.x];
    if (threadIdx.x == 0) {
        int mb = s_max[0];
        for (int w2 = 1; w2 < kWaves; ++w2) mb = s_max[w2] > mb ? s_max[w2] : mb;
        row[kLevels] = mb;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hdr[0] = n_nodes;
        hdr[2] = ioff[P.n];   // inner nodes
    }
}

// Entries at level k of the shared-digit minima (k = -1: the counts
// themselves), each covering 16^(k + 1) positions; INT_MAX past the end.
__device__ __forceinline__ int cd_level(int64_t n, const int32_t* __restrict__ cd, const CdMin& M, int k,
                                        int64_t j) {
    if (k < 0) return j < n ? cd[j] : INT_MAX;
    const int64_t span = (int64_t)1 << (4 * (k + 1));
    return j < (n + span - 1) / span ? M.lev[k][j] : INT_MAX;
}

// next_below for a group of 16 lanes (lane s = 0..15 of the group; every
// lane of the group takes the same path): climb from q, reading at each
// level the entries up to the next boundary of the level above (all of them
// start at or after the positions already passed), until one holds a count
// below l; then descend through its 16 children per level.  About two loads
// per level of the distance instead of up to sixteen.
__device__ int64_t next_below16(int64_t n, const int32_t* __restrict__ cd, const CdMin& M, int64_t q, int l,
                                int s) {
    if (q >= n) return n;
    const int gsh = ag_lane() & 48;   // the group's bits in a wave ballot
    int k = -1;
    int64_t cur = q;   // aligned to the span of level k
    int64_t i;
    for (;;) {
        const int sh = 4 * (k + 1);
        const int64_t idx = cur >> sh;
        const int64_t lim = ((idx >> 4) + 1) << 4;
        const int64_t j = idx + s;
        const int v = j < lim ? cd_level(n, cd, M, k, j) : INT_MAX;
        const unsigned hit = (unsigned)(__ballot(v < l) >> gsh) & 0xffffu;
        if (hit) {
            i = idx + __builtin_ctz(hit);
            break;
        }
        cur = lim << sh;
        if (cur >= n) return n;
        if (k < kCdLevels - 1) ++k;   // cur is now aligned to the next level's span
    }
    for (; k >= 0; --k) {
        const int v = cd_level(n, cd, M, k - 1, 16 * i + s);
        const unsigned hit = (unsigned)(__ballot(v < l) >> gsh) & 0xffffu;
        i = 16 * i + __builtin_ctz(hit);   // the minimum below l lies in one of the children
    }
    return i;
}

// Skip and count fields of the nodes k_write_nodes listed: a group of 16
// lanes per entry (p, t) takes the nodes t, t - 1, .. 0 at p, each end found
// from the one below it, the first from the end of the window k_write_nodes
// searched (no shared-digit count there is below the level of node t, so
// none is below the levels above it either).
__global__ void __launch_bounds__(kThreads) k_far_ends(TopoParams P, const int32_t* __restrict__ cd, CdMin M,
                                                       const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ far_p,
                                                       const int32_t* __restrict__ far_t,
                                                       const int64_t* __restrict__ hdr, int4* __restrict__ link) {
    const int64_t nq = hdr[3];
    const int64_t n_nodes = off[P.n];
    const int s = threadIdx.x & 15;
    for (int64_t g = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 4; g < nq;
         g += ((int64_t)gridDim.x * blockDim.x) >> 4) {
        const int64_t p = far_p[g];
        const int c = cd[p];
        int64_t e = (p & ~(int64_t)63) + kWaveWin;   // the end of the wave's window
        for (int t = far_t[g]; t >= 0; --t) {
            e = next_below16(P.n, cd, M, e, c + 1 + t, s);
            if (s == 0) {
                int4* L = link + off[p] + t;
                L->x = (int)(e < P.n ? (int64_t)off[e] : n_nodes);
                L->z = (int)(e - p);
            }
        }
    }
}

// One block closes the topology: the inner nodes per level and hdr[1] =
// deepest level (from the per-workgroup rows of k_write_nodes), the end of
// the leaves' start list, and the root node of every system.
__global__ void k_tree_close(int nblk, const int32_t* __restrict__ blk, int64_t* __restrict__ hdr,
                             int32_t* __restrict__ leaf_pos, int64_t n, int n_sys,
                             int sys_levels, const int64_t* __restrict__ off, const int32_t* __restrict__ cd,
                             const int32_t* __restrict__ noff, int32_t* __restrict__ root) {
    __shared__ int s_sum[kLevels + 1][16];
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int v[kLevels + 1];
#pragma unroll
    for (int l = 0; l <= kLevels; ++l) v[l] = 0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {   // a row per thread: its loads all in flight
        const int32_t* row = blk + (int64_t)b * (kLevels + 1);
#pragma unroll
        for (int l = 0; l < kLevels; ++l) v[l] += row[l];
        v[kLevels] = row[kLevels] > v[kLevels] ? row[kLevels] : v[kLevels];
    }
#pragma unroll
    for (int l = 0; l <= kLevels; ++l) {
        const int r = l < kLevels ? ag_wave_sum(v[l]) : ag_wave_max(v[l]);
        if ((threadIdx.x & 63) == 0) s_sum[l][w] = r;
    }
    __syncthreads();
    if (threadIdx.x <= kLevels) {
        const int l = threadIdx.x;
        int t = 0;
        for (int k = 0; k < nw; ++k) t = l < kLevels ? t + s_sum[l][k] : (s_sum[l][k] > t ? s_sum[l][k] : t);
        if (l < kLevels) reinterpret_cast<int32_t*>(hdr + 8)[kLvlCnt + l] = t;
        else hdr[1] = t;
    }
    if (threadIdx.x == 0) leaf_pos[hdr[0] - hdr[2]] = (int32_t)n;
    for (int s = threadIdx.x; s < n_sys; s += blockDim.x) {
        const int64_t p0 = off[s];
        if (off[s + 1] <= p0) {
            root[s] = -1;
            continue;
        }
        root[s] = noff[p0] + (sys_levels - cd[p0] - 1);
    }
}

// ---------------------------------------------------------------------------
// 6. moments
// ---------------------------------------------------------------------------
// nd_64 layout per node (25 doubles): M, c(3), u(3), Q(6), Qd(6), lo(3), hi(3)
constexpr int kM64 = 25;

struct NodeOut {
    double4* com;
    float4* lo4;
    float4* hi4;
    float4* mp;
    double* m64;
    const float* sh;   // sorted softening lengths, or null
};

__device__ __forceinline__ uint4 u4_d2(double a, double b) {
    const unsigned long long x = (unsigned long long)__double_as_longlong(a);
    const unsigned long long y = (unsigned long long)__double_as_longlong(b);
    return make_uint4((unsigned)x, (unsigned)(x >> 32), (unsigned)y, (unsigned)(y >> 32));
}
__device__ __forceinline__ uint4 u4_f4(float a, float b, float c, float d) {
    return make_uint4(__float_as_uint(a), __float_as_uint(b), __float_as_uint(c), __float_as_uint(d));
}

// Writes node id's record from a group of G lanes (aligned to G, all
// active) that all hold it (lane s = 0..G-1), so that each store instruction
// writes whole runs: the 25 FP64 moments as runs of G doubles, and the FP32
// copies as 16-byte words, word s of every G (centre of mass and extent in
// two, box low, box high, the four packed multipole words).  lo4.w holds the
// largest softening length in the node (0 without per-particle softening),
// hi4.w the mass.
template <int G>
__device__ __forceinline__ void store_node_g(int64_t id, int s, const double* r, const NodeOut& O, float hmax) {
    // the lane's words are picked by masks, not by indexing or selects on
    // s, which the compiler would turn into an indexed copy in scratch
    unsigned long long mk[G];
#pragma unroll
    for (int k = 0; k < G; ++k) mk[k] = 0ull - (unsigned long long)(s == k);
    double* o = O.m64 + id * kM64;
#pragma unroll
    for (int b = 0; b < kM64; b += G) {
        unsigned long long v = 0ull;
#pragma unroll
        for (int k = 0; k < G; ++k)
            if (b + k < kM64) v |= (unsigned long long)__double_as_longlong(r[b + k]) & mk[k];
        if (b + s < kM64) o[b + s] = __longlong_as_double((long long)v);
    }
    double L = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double e = r[22 + c] - r[19 + c];
        L = e > L ? e : L;
    }
    const uint4 w[8] = {u4_d2(r[1], r[2]),
                        u4_d2(r[3], L),
                        u4_f4(f_down(r[19]), f_down(r[20]), f_down(r[21]), hmax),
                        u4_f4(f_up(r[22]), f_up(r[23]), f_up(r[24]), (float)r[0]),
                        u4_f4((float)r[0], (float)r[4], (float)r[5], (float)r[6]),
                        u4_f4((float)r[7], (float)r[8], (float)r[9], (float)r[10]),
                        u4_f4((float)r[11], (float)r[12], (float)r[13], (float)r[14]),
                        u4_f4((float)r[15], (float)r[16], (float)r[17], (float)r[18])};
#pragma unroll
    for (int b = 0; b < 8; b += G) {
        uint4 val = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const unsigned m = (unsigned)mk[k];
            val.x |= w[b + k].x & m;
            val.y |= w[b + k].y & m;
            val.z |= w[b + k].z & m;
            val.w |= w[b + k].w & m;
        }
        const int wi = b + s;
        uint4* dst = wi < 2 ? reinterpret_cast<uint4*>(O.com + id) + wi
                   : wi == 2 ? reinterpret_cast<uint4*>(O.lo4 + id)
                   : wi == 3 ? reinterpret_cast<uint4*>(O.hi4 + id)
                             : reinterpret_cast<uint4*>(O.mp + 4 * id) + (wi - 4);
        *dst = val;
    }
}

// Q  += m (3 y y^T - |y|^2 I),  Qd += m (3 (y w^T + w y^T) - 2 (y.w) I)
__device__ __forceinline__ void add_quad(double* Q, double* Qd, double mm, const double* y, const double* w) {
    const double y2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    const double yw = y[0] * w[0] + y[1] * w[1] + y[2] * w[2];
    const int a[6] = {0, 1, 2, 0, 0, 1}, b[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double del = k < 3 ? 1.0 : 0.0;
        Q[k] += mm * (3.0 * y[a[k]] * y[b[k]] - y2 * del);
        Qd[k] += mm * (3.0 * (y[a[k]] * w[b[k]] + w[a[k]] * y[b[k]]) - 2.0 * yw * del);
    }
}

// One-pass accumulation of the moments of a set of point masses (particles,
// or children's centres of mass carrying their own Q and Qd): positions and
// velocities are taken relative to the first member (r0, u0), and the sums
// are moved to the centre of mass at the end with the parallel-axis rule
//   sum m (3 y y^T - y^2 I) = sum m (3 e e^T - e^2 I) - M (3 E E^T - E^2 I),
// y = e - E, E = sum m e / M (and the same bilinear rule for Qd).
struct MomentSums {
    double r0[3], u0[3];
    double M, e[3], f[3];         // mass, sum m e, sum m f (e = x - r0, f = u - u0)
    double Q[6], Qd[6];           // about r0, u0 (plus the members' own Q, Qd)
    double lo[3], hi[3];
    bool first;
    __device__ void init() {
        M = 0.0;
        for (int c = 0; c < 3; ++c) {
            e[c] = f[c] = 0.0;
            lo[c] = DBL_MAX;
            hi[c] = -DBL_MAX;
        }
        for (int k = 0; k < 6; ++k) Q[k] = Qd[k] = 0.0;
        first = true;
    }
    __device__ void add(double m, const double* x, const double* u) {
        if (first) {
            for (int c = 0; c < 3; ++c) { r0[c] = x[c]; u0[c] = u[c]; }
            first = false;
        }
        const double ee[3] = {x[0] - r0[0], x[1] - r0[1], x[2] - r0[2]};
        const double ff[3] = {u[0] - u0[0], u[1] - u0[1], u[2] - u0[2]};
        M += m;
        for (int c = 0; c < 3; ++c) {
            e[c] += m * ee[c];
            f[c] += m * ff[c];
        }
        add_quad(Q, Qd, m, ee, ff);
    }
    __device__ void box(const double* l, const double* h) {
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], l[c]);
            hi[c] = fmax(hi[c], h[c]);
        }
    }
    // r: M, c(3), u(3), Q(6), Qd(6), lo(3), hi(3)
    __device__ void finish(double* r) const {
        r[0] = M;
        // branch-free (a massless cell takes the centre of its box and
        // velocity zero), which keeps r in registers
        const bool pos = M > 0.0;
        const double Mi = pos ? 1.0 / M : 0.0;
        double E[3], F[3];
        for (int c = 0; c < 3; ++c) {
            r[19 + c] = lo[c];
            r[22 + c] = hi[c];
            E[c] = e[c] * Mi;
            F[c] = f[c] * Mi;
            r[1 + c] = pos ? r0[c] + E[c] : 0.5 * (lo[c] + hi[c]);
            r[4 + c] = pos ? u0[c] + F[c] : 0.0;
        }
        double q[6], qd[6];
        for (int k = 0; k < 6; ++k) q[k] = qd[k] = 0.0;
        add_quad(q, qd, M, E, F);
        for (int k = 0; k < 6; ++k) {
            r[7 + k] = Q[k] - q[k];
            r[13 + k] = Qd[k] - qd[k];
        }
    }
};

// Reductions over the G lanes of a group (G = 2, 4 or 8, aligned to G,
// all active) by DPP moves, which stay in the vector unit (no LDS
// permutes): partners at xor 1 and xor 2 within each quad, then the mirror
// lane within each eight (lane 7 - i, which is in the other quad).  Every
// lane ends with the same bits: each step adds two values that are equal on
// both partners.
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror
template <int C> __device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, C, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), C, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int C> __device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), C, 0xF, 0xF, false));
}
template <int G> __device__ __forceinline__ double grp_sum(double v) {
    if (G >= 2) v += dpp_f64<kDppXor1>(v);
    if (G >= 4) v += dpp_f64<kDppXor2>(v);
    if (G >= 8) v += dpp_f64<kDppHalfMirror>(v);
    return v;
}
template <int G> __device__ __forceinline__ double grp_min(double v) {
    if (G >= 2) v = fmin(v, dpp_f64<kDppXor1>(v));
    if (G >= 4) v = fmin(v, dpp_f64<kDppXor2>(v));
    if (G >= 8) v = fmin(v, dpp_f64<kDppHalfMirror>(v));
    return v;
}
template <int G> __device__ __forceinline__ double grp_max(double v) {
    if (G >= 2) v = fmax(v, dpp_f64<kDppXor1>(v));
    if (G >= 4) v = fmax(v, dpp_f64<kDppXor2>(v));
    if (G >= 8) v = fmax(v, dpp_f64<kDppHalfMirror>(v));
    return v;
}
template <int G> __device__ __forceinline__ float grp_maxf(float v) {
    if (G >= 2) v = fmaxf(v, dpp_f32<kDppXor1>(v));
    if (G >= 4) v = fmaxf(v, dpp_f32<kDppXor2>(v));
    if (G >= 8) v = fmaxf(v, dpp_f32<kDppHalfMirror>(v));
    return v;
}
template <int G> __device__ __forceinline__ void grp_reduce(MomentSums& S) {
    S.M = grp_sum<G>(S.M);
    for (int c = 0; c < 3; ++c) {
        S.e[c] = grp_sum<G>(S.e[c]);
        S.f[c] = grp_sum<G>(S.f[c]);
        S.lo[c] = grp_min<G>(S.lo[c]);
        S.hi[c] = grp_max<G>(S.hi[c]);
    }
    for (int k = 0; k < 6; ++k) {
        S.Q[k] = grp_sum<G>(S.Q[k]);
        S.Qd[k] = grp_sum<G>(S.Qd[k]);
    }
}

// For every inner node: its place in the list of inner nodes grouped by
// level (order within a level is immaterial: every block ranks its nodes per
// level in LDS and takes one slot range per level with a global atomic;
// block 0 also writes the level offsets), where the slot receives the node's
// id and, in the child rows, its children by octant (-1 where an octant is
// empty), from the pre-order links (the first child follows the node, the
// next follows the first child's subtree, ...).  A level's kernels then read
// a node and its children from the same slot.
__global__ void __launch_bounds__(kThreads) k_level_lists(const int64_t* __restrict__ hdr,
                                                          const int32_t* __restrict__ ilist,
                                                          const int4* __restrict__ link,
                                                          const uint64_t* __restrict__ keys,
                                                          int4* __restrict__ child,
                                                          int32_t* __restrict__ lvl,
                                                          int32_t* __restrict__ lvl_list) {
    __shared__ int s_off[AG_MAX_LEVEL + 2], s_cnt[AG_MAX_LEVEL + 1], s_base[AG_MAX_LEVEL + 1];
    const int64_t ni = hdr[2];
    if (threadIdx.x == 0) {
        int a = 0;
        for (int l = 0; l <= AG_MAX_LEVEL; ++l) {
            s_off[l] = a;
            a += lvl[kLvlCnt + l];
        }
        s_off[AG_MAX_LEVEL + 1] = a;
    }
    if (threadIdx.x <= AG_MAX_LEVEL) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x <= AG_MAX_LEVEL + 1) lvl[kLvlOff + threadIdx.x] = s_off[threadIdx.x];
    for (int64_t t0 = (int64_t)blockIdx.x * kThreads; t0 < ni; t0 += (int64_t)gridDim.x * kThreads) {
        const int64_t t = t0 + threadIdx.x;
        int node = -1, l = 0, r = 0;
        int c8[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
        if (t < ni) {
            node = ilist[t];
            const int4 L = link[node];
            l = L.w & 0xff;
            r = atomicAdd(&s_cnt[l], 1);
            const int sh = 63 - 3 * (l + 1);   // the children's own octal digit
            for (int ch = node + 1, k8 = 0; ch < L.x && k8 < 8; ++k8) {
                const int4 C = link[ch];
                c8[(int)((keys[C.y] >> sh) & 7)] = ch;
                ch = C.x;
            }
        }
        __syncthreads();
        if (threadIdx.x <= AG_MAX_LEVEL && s_cnt[threadIdx.x] > 0) {
            s_base[threadIdx.x] = atomicAdd(&lvl[kLvlCur + threadIdx.x], s_cnt[threadIdx.x]);
            s_cnt[threadIdx.x] = 0;
        }
        __syncthreads();
        if (node >= 0) {
            const int64_t slot = s_off[l] + s_base[l] + r;
            lvl_list[slot] = node;
            child[2 * slot] = make_int4(c8[0], c8[1], c8[2], c8[3]);
            child[2 * slot + 1] = make_int4(c8[4], c8[5], c8[6], c8[7]);
        }
        __syncthreads();
    }
}

// Forms inner node id (child row in) from its children with a group of G
// lanes (aligned to G, all active), lane s taking octants s, s + G, ...:
// each lane forms its children's terms about the first child's centre of
// mass and velocity, and the lanes sum them by DPP moves.
template <int G>
__device__ void form_inner(int in, int id, int s, const int32_t* __restrict__ child, const NodeOut& O) {
    const int4 ca = reinterpret_cast<const int4*>(child)[2 * (int64_t)in];
    const int4 cb = reinterpret_cast<const int4*>(child)[2 * (int64_t)in + 1];
    const int c8[8] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
    int chf = -1;   // the first octant that holds a child supplies the reference point
#pragma unroll
    for (int k = 7; k >= 0; --k) chf = c8[k] >= 0 ? c8[k] : chf;
    MomentSums S;
    S.init();
    for (int c = 0; c < 3; ++c) {
        S.r0[c] = chf >= 0 ? O.m64[(int64_t)chf * kM64 + 1 + c] : 0.0;
        S.u0[c] = chf >= 0 ? O.m64[(int64_t)chf * kM64 + 4 + c] : 0.0;
    }
    S.first = false;
    float hm = 0.f;
#pragma unroll
    for (int j = 0; j < 8 / G; ++j) {
        int ch = 0;   // c8[s + j G], picked by masks (no indexing by the lane number)
#pragma unroll
        for (int k = 0; k < 8; ++k) ch |= c8[k] & -(int)(k == s + j * G);
        if (ch >= 0) {
            const double* cm = O.m64 + (int64_t)ch * kM64;
            S.add(cm[0], cm + 1, cm + 4);
            for (int k = 0; k < 6; ++k) {
                S.Q[k] += cm[7 + k];
                S.Qd[k] += cm[13 + k];
            }
            S.box(cm + 19, cm + 22);
            hm = fmaxf(hm, O.lo4[ch].w);
        }
    }
    grp_reduce<G>(S);
    hm = grp_maxf<G>(hm);
    double r[kM64];
    S.finish(r);
    store_node_g<G>(id, s, r, O, hm);
}

// Every leaf from its particles: a group of kLeafLanes lanes per leaf (leaf
// list order, so a wave reads a contiguous run of particles), each lane
// summing every kLeafLanes-th particle about the leaf's first one, the sums
// added across the group by DPP moves and the record written by the whole
// group.  The velocities are read from the caller's array through the
// sorted rows (perm: position -> input row); their FP32 copies, with the
// masses (for the walk), are written here in order.
constexpr int kLeafLanes = 4;
constexpr int kInnerLanes = 8;
__global__ void __launch_bounds__(kThreads) k_leaf_moments(const int64_t* __restrict__ hdr,
                                                           const int32_t* __restrict__ leaves,
                                                           const int32_t* __restrict__ leaf_pos,
                                                           const double4* __restrict__ spos,
                                                           const int32_t* __restrict__ perm,
                                                           const double* __restrict__ v,
                                                           float4* __restrict__ svf, NodeOut O) {
    constexpr int G = kLeafLanes;
    const int64_t nl = hdr[0] - hdr[2];
    const int s = threadIdx.x & (G - 1);
    const int64_t stride = ((int64_t)gridDim.x * blockDim.x) / G;
    for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G; g < nl; g += stride) {
        const int id = leaves[g];
        const int p0 = leaf_pos[g], p1 = leaf_pos[g + 1];   // the leaves cover the positions in order
        MomentSums S;
        S.init();
        {
            const double4 a = spos[p0];
            const int64_t r = perm[p0];
            S.r0[0] = a.x; S.r0[1] = a.y; S.r0[2] = a.z;
            S.u0[0] = v[3 * r]; S.u0[1] = v[3 * r + 1]; S.u0[2] = v[3 * r + 2];
            S.first = false;
        }
        float hm = 0.f;
        for (int q = p0 + s; q < p1; q += G) {
            const double4 a = spos[q];
            const int64_t r = perm[q];
            const double u[3] = {v[3 * r], v[3 * r + 1], v[3 * r + 2]};
            svf[q] = make_float4((float)u[0], (float)u[1], (float)u[2], (float)a.w);
            const double x[3] = {a.x, a.y, a.z};
            S.add(a.w, x, u);
            S.box(x, x);
            if (O.sh) hm = fmaxf(hm, O.sh[q]);
        }
        grp_reduce<G>(S);
        hm = grp_maxf<G>(hm);
        double r[kM64];
        S.finish(r);
        store_node_g<G>(id, s, r, O, hm);
    }
}

// Inner nodes of levels l_hi down to l_lo from their children, kInnerLanes
// lanes per node: one level per launch (l_hi = l_lo, any grid; launched from the
// deepest up, so every child is complete when its parent is formed), or
// several in a single-workgroup launch, the workgroup barrier between levels
// ordering each level after its children's.
__global__ void __launch_bounds__(kThreads) k_inner_level(int l_hi, int l_lo, const int32_t* __restrict__ lvl,
                                                          const int32_t* __restrict__ lvl_list,
                                                          const int32_t* __restrict__ child, NodeOut O) {
    constexpr int G = kInnerLanes;
    const int s = threadIdx.x & (G - 1);
    const int64_t slot = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int64_t nslot = ((int64_t)gridDim.x * blockDim.x) / G;
    for (int level = l_hi; level >= l_lo; --level) {
        if (level < l_hi) __syncthreads();   // single-workgroup launches only
        const int t_lo = lvl[kLvlOff + level], t_hi = lvl[kLvlOff + level + 1];
        for (int64_t t = t_lo + slot; t < t_hi; t += nslot)   // uniform over the group
            form_inner<G>((int)t, lvl_list[t], s, child, O);
    }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Moments: the leaves, then the inner levels from the deepest up.  The
// levels below the deepest of the last build whose depth the host has seen
// (c->seen_max_level; 20 if none) take one single-workgroup launch (they are
// usually empty), the levels from there to 3 one launch each, and levels 2-0
// (at most 73 nodes) one single-workgroup launch.  A deeper tree than
// expected is still complete, only slower.
int moments_pass(ag_ctx* c, const double* v) {
    hipStream_t st = c->stream;
    NodeOut O{c->nd_com.as<double4>(), c->nd_lo.as<float4>(), c->nd_hi.as<float4>(), c->nd_mp.as<float4>(),
              c->nd_64.as<double>(), c->tree_soft ? c->soft_s.as<float>() : nullptr};
    const int64_t n = c->n;
    hipLaunchKernelGGL(k_leaf_moments, dim3(grid_for(kLeafLanes * n)), dim3(kThreads), 0, st, c->tree_hdr.as<int64_t>(),
                       c->leaf_list.as<int32_t>(), c->leaf_pos.as<int32_t>(), c->spos.as<double4>(),
                       c->perm.as<int32_t>(), v, c->svf.as<float4>(), O);
    // level-21 cells are always leaves; empty levels exit at once
    const int64_t inner_bound = c->max_nodes - n;
    int g = grid_for(kInnerLanes * (inner_bound > 0 ? inner_bound : 1));
    if (g > 1024) g = 1024;
    const int32_t* lvl = reinterpret_cast<const int32_t*>(c->tree_hdr.as<int64_t>() + 8);
    constexpr int kTop = 2;
    int lc = c->seen_max_level - 1;   // inner nodes lie above the deepest level
    if (c->seen_max_level < 0 || lc > AG_MAX_LEVEL - 1) lc = AG_MAX_LEVEL - 1;
    if (lc < kTop + 1) lc = kTop;
    const int32_t* ll = c->lvl_list.as<int32_t>();
    const int32_t* ch = c->child.as<int32_t>();
    if (lc < AG_MAX_LEVEL - 1)
        hipLaunchKernelGGL(k_inner_level, dim3(1), dim3(kThreads), 0, st, AG_MAX_LEVEL - 1, lc + 1, lvl, ll, ch, O);
    for (int l = lc; l > kTop; --l)
        hipLaunchKernelGGL(k_inner_level, dim3(g), dim3(kThreads), 0, st, l, l, lvl, ll, ch, O);
    hipLaunchKernelGGL(k_inner_level, dim3(1), dim3(kThreads), 0, st, kTop, 0, lvl, ll, ch, O);
    return AG_OK;
}

}  // namespace

int ag_launch_build(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m, int32_t n_sys,
                    const int64_t* sys_offsets, int32_t n_leaf) {
    int sys_levels = 0;
    if (sys_offsets) {
        while ((1 << (3 * sys_levels)) < n_sys) ++sys_levels;
        if (sys_levels < 1) sys_levels = 1;
    }
    const int bits = AG_MAX_LEVEL - sys_levels;
    // leaves <= n; at each level the split cells are disjoint and hold more
    // than n_leaf particles (or are system-prefix cells)
    const int64_t max_nodes = n + (int64_t)(AG_MAX_LEVEL + 1) * (n / (n_leaf + 1) + n_sys) + 1;

    AG_TRY(ag_ensure(c, c->keys[0], n * 8)); AG_TRY(ag_ensure(c, c->keys[1], n * 8));
    AG_TRY(ag_ensure(c, c->vals[0], n * 4)); AG_TRY(ag_ensure(c, c->vals[1], n * 4));
    const int nblocks = (int)((n + kRsTile - 1) / kRsTile);
    // (also the bounding boxes' per-workgroup partials before the sort, and
    // k_write_nodes' per-workgroup rows after it)
    const int wblocks = std::min(grid_for(n), kWriteBlocks);
    AG_TRY(ag_ensure(c, c->sort_hist, std::max({(size_t)(256 * nblocks + 256 + 1) * 4,
                                                (size_t)(n / kBoxChunk + n_sys + 1) * 6 * sizeof(uint64_t),
                                                (size_t)wblocks * (kLevels + 1) * sizeof(int32_t)})));
    AG_TRY(ag_ensure(c, c->pos_off, (size_t)(256 * (int64_t)nblocks + 1 > n + 1 ? 256 * (int64_t)nblocks + 1 : n + 1) * 4));
    AG_TRY(ag_ensure(c, c->perm, n * 4)); AG_TRY(ag_ensure(c, c->rank, n * 4));
    AG_TRY(ag_ensure(c, c->spos, n * 32)); AG_TRY(ag_ensure(c, c->svf, n * 16));
    AG_TRY(ag_ensure(c, c->cdig, n * 4)); AG_TRY(ag_ensure(c, c->pos_cnt, (n + 1) * 4));
    // minima of the shared-digit counts: level 0 per 16 positions (16 per run of
    // 256), levels k >= 1 per 16^(k+1)
    int64_t cd_cnt[kCdLevels], cd_tot = 0;
    const int64_t passes = (n + kCdPass - 1) / kCdPass;   // k_cdig writes levels 0-2 for whole passes
    cd_cnt[0] = passes * 256;
    cd_cnt[1] = passes * 16;
    cd_cnt[2] = passes;
    for (int k = 3; k < kCdLevels; ++k) {
        const int64_t span = (int64_t)1 << (4 * (k + 1));
        cd_cnt[k] = (n + span - 1) / span;
    }
    for (int k = 0; k < kCdLevels; ++k) cd_tot += cd_cnt[k];
    AG_TRY(ag_ensure(c, c->cd_min, (size_t)cd_tot * sizeof(int32_t)));
    AG_TRY(ag_ensure(c, c->nd_com, max_nodes * 32)); AG_TRY(ag_ensure(c, c->nd_lo, max_nodes * 16));
    AG_TRY(ag_ensure(c, c->nd_hi, max_nodes * 16)); AG_TRY(ag_ensure(c, c->nd_link, max_nodes * 16));
    AG_TRY(ag_ensure(c, c->nd_mp, max_nodes * 64)); AG_TRY(ag_ensure(c, c->nd_64, max_nodes * kM64 * 8));
    AG_TRY(ag_ensure(c, c->in_list, max_nodes * 4)); AG_TRY(ag_ensure(c, c->in_cnt, (n + 1) * 4));
    AG_TRY(ag_ensure(c, c->in_off, (n + 1) * 4));
    AG_TRY(ag_ensure(c, c->sys_off, (n_sys + 1) * 8)); AG_TRY(ag_ensure(c, c->sys_root, (n_sys + 1) * 4));
    const int64_t inner_bound = max_nodes - n;   // inner nodes never exceed this
    AG_TRY(ag_ensure(c, c->lvl_list, (size_t)(inner_bound > 0 ? inner_bound : 1) * 4));
    AG_TRY(ag_ensure(c, c->leaf_list, n * 4));   // at most one leaf starts at each position
    AG_TRY(ag_ensure(c, c->leaf_pos, (n + 1) * 4));
    AG_TRY(ag_ensure(c, c->child, (size_t)(inner_bound > 0 ? inner_bound : 1) * 32));
    AG_TRY(ag_ensure(c, c->sys_box, 6 * n_sys * 8 + 8 * (n_sys + 1)));

    if (c->depth_pending && !c->capturing && hipEventQuery(c->depth_ev) == hipSuccess) {
        c->seen_max_level = (int)*c->depth_host;
        c->depth_pending = false;
    }

    PhaseScope phase(c, AG_PHASE_BUILD);
    hipStream_t st = c->stream;
    int32_t* flags = c->dflags.as<int32_t>();
    int64_t* off = c->sys_off.as<int64_t>();
    int64_t* hdr = c->tree_hdr.as<int64_t>();

    // 1. bounding cubes
    uint64_t* box = c->sys_box.as<uint64_t>();
    int32_t* blk_off = reinterpret_cast<int32_t*>(box + 6 * n_sys);
    CdMin M;
    {
        int32_t* q = c->cd_min.as<int32_t>();
        for (int k = 0; k < kCdLevels; ++k) {
            M.lev[k] = q;
            q += cd_cnt[k];
        }
    }
    hipLaunchKernelGGL(k_build_init, dim3(1), dim3(512), 0, st, n_sys, n, sys_offsets, off, flags, box, blk_off, hdr,
                       (int)(kTreeHdrBytes / 8));
    const int64_t box_blocks = n / kBoxChunk + n_sys + 1;
    uint64_t* box_part = reinterpret_cast<uint64_t*>(c->sort_hist.p);   // free until the sort
    hipLaunchKernelGGL(k_box, dim3((unsigned)box_blocks), dim3(kBoxThreads), 0, st, x, off, n_sys, blk_off, box_part,
                       flags, c->box);
    hipLaunchKernelGGL(k_box_reduce, dim3((unsigned)n_sys), dim3(256), 0, st, n_sys, blk_off, box_part, box);

    // 2. keys
    uint64_t* k0 = c->keys[0].as<uint64_t>();
    uint64_t* k1 = c->keys[1].as<uint64_t>();
    int32_t* v0 = c->vals[0].as<int32_t>();
    int32_t* v1 = c->vals[1].as<int32_t>();
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n)), dim3(kThreads), 0, st, n, x, off, n_sys, bits, box, k0, v0, c->box);

    // 3. sort: four passes over bits 31..62 (the last writes the permutation
    //    and its inverse), then the level-10 cells holding more than n_leaf
    //    particles by their full keys
    int32_t* hist = c->sort_hist.as<int32_t>();
    int32_t* tot = hist + (int64_t)256 * nblocks;
    int32_t* hoff = c->pos_off.as<int32_t>();
    int32_t* perm = c->perm.as<int32_t>();
    int32_t* rank = c->rank.as<int32_t>();
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = kSortedShift + 8 * pass;
        uint64_t* kin = (pass & 1) ? k1 : k0;
        uint64_t* kout = (pass & 1) ? k0 : k1;
        int32_t* vin = (pass & 1) ? v1 : v0;
        int32_t* vout = pass == 3 ? perm : ((pass & 1) ? v0 : v1);
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(kThreads), 0, st, kin, n, shift, nblocks, hist);
        hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(kThreads), 0, st, hist, nblocks, hoff, tot);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(kThreads), 0, st, kin, vin, n, shift, nblocks, hist,
                           hoff, tot, kout, vout, pass == 3 ? rank : (int32_t*)nullptr);
    }
    {
        TopoParams PS{n, n_leaf, sys_levels};
        int32_t* flag = c->pos_cnt.as<int32_t>();   // free until the topology
        int32_t* soff = c->pos_off.as<int32_t>();
        int32_t* list = c->cdig.as<int32_t>();
        hipLaunchKernelGGL(k_seg_heads, dim3(grid_for(n)), dim3(kThreads), 0, st, n, k0, n_leaf, flag);
        AG_TRY(ag_scan_i32(c, flag, soff, n));
        hipLaunchKernelGGL(k_seg_list, dim3(grid_for(n)), dim3(kThreads), 0, st, n, flag, soff, list);
        const int64_t cells = n / (n_leaf + 1) + 1;   // dense cells are disjoint and hold > n_leaf each
        hipLaunchKernelGGL(k_seg_sort, dim3((unsigned)(cells < 2048 ? cells : 2048)), dim3(kThreads), 0, st, PS,
                           list, soff + n, k0, perm, rank, k1, v1);
    }

    // 4. particle data into key order
    c->tree_soft = c->soft_n > 0;
    if (c->tree_soft) AG_TRY(ag_ensure(c, c->soft_s, (size_t)n * sizeof(float)));
    launch_to_sorted(c, n, x, m, c->box);
    c->tree_box = c->box;

    // 5. topology
    int32_t* cd = c->cdig.as<int32_t>();
    {
        int64_t cb = passes < 4096 ? passes : 4096;
        hipLaunchKernelGGL(k_cdig, dim3((unsigned)cb), dim3(kRun), 0, st, n, k0, cd, M);
        CdCounts C;
        for (int k = 0; k < kCdLevels; ++k) C.cnt[k] = cd_cnt[k];
        hipLaunchKernelGGL(k_cd_min_top, dim3(1), dim3(1024), 0, st, M, C);
    }
    TopoParams P{n, n_leaf, sys_levels};
    int32_t* pcnt = c->pos_cnt.as<int32_t>();
    int32_t* poff = c->pos_off.as<int32_t>();
    int32_t* icnt = c->in_cnt.as<int32_t>();
    int32_t* ioff = c->in_off.as<int32_t>();
    hipLaunchKernelGGL(k_count_nodes, dim3(grid_for(n)), dim3(kThreads), 0, st, P, cd, pcnt, icnt);
    AG_TRY(ag_scan_i32(c, pcnt, poff, n));
    AG_TRY(ag_scan_i32(c, icnt, ioff, n));
    // (the node counts are free after their scans: they hold the list of far
    // ends; the sort's histograms hold the per-workgroup rows)
    int32_t* blk_rows = c->sort_hist.as<int32_t>();
    hipLaunchKernelGGL(k_write_nodes, dim3(wblocks), dim3(kThreads), 0, st, P, cd, poff, ioff,
                       c->nd_link.as<int4>(), c->in_list.as<int32_t>(), c->leaf_list.as<int32_t>(),
                       c->leaf_pos.as<int32_t>(), hdr, blk_rows,
                       pcnt, icnt);
    hipLaunchKernelGGL(k_far_ends, dim3(grid_for(n / 16 + 1)), dim3(kThreads), 0, st, P, cd, M, poff, pcnt, icnt,
                       hdr, c->nd_link.as<int4>());
    hipLaunchKernelGGL(k_tree_close, dim3(1), dim3(1024), 0, st, wblocks, blk_rows, hdr, c->leaf_pos.as<int32_t>(),
                       n, n_sys, sys_levels, off, cd,
                       poff, c->sys_root.as<int32_t>());
    if (!c->capturing && c->depth_host) {   // this tree's depth, for the next build's launch plan
        (void)hipMemcpyAsync(c->depth_host, hdr + 1, sizeof(int64_t), hipMemcpyDeviceToHost, st);
        (void)hipEventRecord(c->depth_ev, st);
        c->depth_pending = true;
    }
    hipLaunchKernelGGL(k_level_lists, dim3(grid_for(inner_bound) < 1024 ? grid_for(inner_bound) : 1024),
                       dim3(kThreads), 0, st, hdr, c->in_list.as<int32_t>(), c->nd_link.as<int4>(), k0,
                       c->child.as<int4>(), reinterpret_cast<int32_t*>(hdr + 8), c->lvl_list.as<int32_t>());

    c->n = n;
    c->n_leaf = n_leaf;
    c->n_sys = n_sys;
    c->sys_levels = sys_levels;
    c->max_nodes = max_nodes;

    // 6. moments
    return moments_pass(c, v);
}

int ag_launch_refit(ag_ctx* c, const double* x, const double* v, const double* m) {
    const int64_t n = c->n;
    PhaseScope phase(c, AG_PHASE_BUILD);
    launch_to_sorted(c, n, x, m, c->tree_box);
    return moments_pass(c, v);
}
