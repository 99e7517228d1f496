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
constexpr int64_t kBoxChunk = 8192;

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

__global__ void __launch_bounds__(kThreads) k_box(const double* __restrict__ x, const int64_t* __restrict__ off,
                                                  int n_sys, const int32_t* __restrict__ blk_off,
                                                  uint64_t* __restrict__ box, int32_t* __restrict__ flags,
                                                  double pbox) {
    __shared__ double s_red[6][kThreads / 64];
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
    double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    bool bad = false;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double q = x[3 * i + c];
            if (!isfinite(q)) { bad = true; continue; }
            q = in_box(q, pbox);
            mn[c] = q < mn[c] ? q : mn[c];
            mx[c] = q > mx[c] ? q : mx[c];
        }
    }
    if (bad) atomicOr(flags, AGF_NONFINITE);
    const int lane = ag_lane(), w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double a = ag_wave_min(mn[c]), z = ag_wave_max(mx[c]);
        if (lane == 0) { s_red[c][w] = a; s_red[3 + c][w] = z; }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int c = threadIdx.x;
        double r = s_red[c][0];
        for (int k = 1; k < kThreads / 64; ++k)
            r = c < 3 ? (s_red[c][k] < r ? s_red[c][k] : r) : (s_red[c][k] > r ? s_red[c][k] : r);
        if (c < 3) atomicMin((unsigned long long*)&box[6 * s + c], (unsigned long long)ag_ord(r));
        else atomicMax((unsigned long long*)&box[6 * s + c], (unsigned long long)ag_ord(r));
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
constexpr int kRsItems = 8;
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

// Stable scatter of one tile of (key, value) pairs by one 8-bit digit.  The
// tile is first ranked and reordered by digit in LDS (ballot matching within
// each wave, per-wave counts across the block), then written out in digit
// order so that each digit's run goes to consecutive addresses.  With `rank`
// set (last pass), rank[value] receives the value's final position.
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
    __shared__ int s_run[256];
    __shared__ int s_w[4][256];
    __shared__ int s_tmp[kThreads / 64];
    const int t = threadIdx.x;
    {
        int all;
        const int base_d = block_excl_scan256(tot[t], s_tmp, &all);
        const int loc = block_excl_scan256(hist[(int64_t)t * nblocks + blockIdx.x], s_tmp, &all);
        s_loc[t] = loc;
        s_gofs[t] = base_d + hoff[(int64_t)t * nblocks + blockIdx.x] - loc;
        s_run[t] = 0;
    }
    const int w = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int k = 0; k < kRsItems; ++k) {
        const int64_t i = base + k * kThreads + t;
        const bool valid = i < n;
        const uint64_t key = valid ? kin[i] : 0ull;
        const int32_t val = valid ? vin[i] : 0;
        const int d = (int)((key >> shift) & 255);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const int r = ag_prefix_count(peers);
        const int cnt = __popcll(peers);
#pragma unroll
        for (int q = 0; q < 4; ++q) s_w[q][t] = 0;
        __syncthreads();
        if (valid && r == 0) s_w[w][d] = cnt;
        __syncthreads();
        {
            int run = s_run[t];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int c = s_w[q][t];
                s_w[q][t] = run;
                run += c;
            }
            s_run[t] = run;
        }
        __syncthreads();
        if (valid) {
            const int slot = s_loc[d] + s_w[w][d] + r;
            s_key[slot] = key;
            s_val[slot] = val;
        }
        __syncthreads();
    }
    const int64_t rem = n - base;
    const int nvalid = rem < kRsTile ? (int)rem : kRsTile;
    for (int j = t; j < nvalid; j += kThreads) {
        const uint64_t key = s_key[j];
        const int d = (int)((key >> shift) & 255);
        const int pos = s_gofs[d] + j;
        kout[pos] = key;
        const int32_t val = s_val[j];
        vout[pos] = val;
        if (rank) rank[val] = pos;
    }
}

// ---------------------------------------------------------------------------
// 4. particle data into key order: coalesced reads in input order, each row
//    written to its sorted position (scattered 32-byte stores)
// ---------------------------------------------------------------------------
__global__ void k_to_sorted(int64_t n, const int32_t* __restrict__ rank, const double* __restrict__ x,
                            const double* __restrict__ v, const double* __restrict__ m,
                            double4* __restrict__ spos, double4* __restrict__ svel, float4* __restrict__ svf,
                            double pbox, const double* __restrict__ h, float* __restrict__ sh) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = rank[i];
        const double mi = m[i];
        const double vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
        spos[p] = make_double4(in_box(x[3 * i], pbox), in_box(x[3 * i + 1], pbox), in_box(x[3 * i + 2], pbox), mi);
        svel[p] = make_double4(vx, vy, vz, 0.0);
        svf[p] = make_float4((float)vx, (float)vy, (float)vz, (float)mi);
        if (h) sh[p] = f_up(h[i]);   // per-particle softening, rounded up
    }
}

// ---------------------------------------------------------------------------
// 5. topology
// ---------------------------------------------------------------------------
__device__ __forceinline__ int common_digits(uint64_t a, uint64_t b) {
    const uint64_t d = a ^ b;
    if (d == 0) return AG_MAX_LEVEL;
    return (__clzll(d) - 1) / 3;   // bit 63 is always clear
}

__global__ void k_cdig(int64_t n, const uint64_t* __restrict__ keys, int32_t* __restrict__ cd) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        cd[p] = p == 0 ? -1 : common_digits(keys[p - 1], keys[p]);
}

struct TopoParams {
    int64_t n;
    int n_leaf;
    int sys_levels;
};

__device__ __forceinline__ bool is_split(const TopoParams& P, int level, int64_t count_or_big) {
    if (level < P.sys_levels) return true;
    return level < AG_MAX_LEVEL && count_or_big > P.n_leaf;
}

// end of the level-l cell starting at p if it holds <= n_leaf particles,
// else -1 (bounded forward scan of the shared-digit counts)
__device__ __forceinline__ int64_t small_cell_end(const TopoParams& P, const int32_t* __restrict__ cd,
                                                  int64_t p, int l) {
    int64_t q = p + 1;
    const int64_t lim = p + P.n_leaf;
    while (q < P.n && q <= lim) {
        if (cd[q] < l) return q;
        ++q;
    }
    if (q >= P.n && P.n - p <= P.n_leaf) return P.n;
    return -1;
}

// does the level-c cell containing p (which does not start at p) get split?
__device__ __forceinline__ bool parent_split(const TopoParams& P, const int32_t* __restrict__ cd, int64_t p,
                                             int c) {
    if (c < P.sys_levels) return true;
    if (c >= AG_MAX_LEVEL) return false;
    int64_t a = p - 1;
    int steps = 0;
    while (cd[a] >= c) {       // cd[0] = -1 stops the scan
        --a;
        if (++steps > P.n_leaf) return true;
    }
    int64_t q = p + 1;
    while (q < P.n && cd[q] >= c) {
        ++q;
        if (++steps > P.n_leaf) return true;
    }
    return (q - a) > P.n_leaf;
}

// number of tree nodes starting at position p
__device__ __forceinline__ int nodes_at(const TopoParams& P, const int32_t* __restrict__ cd, int64_t p) {
    const int c = cd[p];
    if (p > 0 && (c >= AG_MAX_LEVEL || !parent_split(P, cd, p, c))) return 0;
    int cnt = 0;
    for (int l = c + 1; l <= AG_MAX_LEVEL; ++l) {
        ++cnt;
        const int64_t e = small_cell_end(P, cd, p, l);
        const bool small = e >= 0;
        if (!is_split(P, l, small ? 0 : P.n_leaf + 1)) break;
    }
    return cnt;
}

// nodes starting at each position, and how many of them are inner nodes
// (all but the last, which is a leaf)
__global__ void k_count_nodes(TopoParams P, const int32_t* __restrict__ cd, int32_t* __restrict__ cnt,
                              int32_t* __restrict__ icnt) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P.n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int k = nodes_at(P, cd, p);
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

// Writes every node's link and lists the inner nodes (in pre-order).
__global__ void k_write_nodes(TopoParams P, const uint64_t* __restrict__ keys, const int32_t* __restrict__ cd,
                              const int32_t* __restrict__ off, const int32_t* __restrict__ ioff,
                              int4* __restrict__ link, int32_t* __restrict__ ilist, int32_t* __restrict__ leaves,
                              int64_t* __restrict__ hdr, int32_t* __restrict__ blk_max) {
    __shared__ int s_lc[AG_MAX_LEVEL + 1];   // inner nodes of this block per level
    if (threadIdx.x <= AG_MAX_LEVEL) s_lc[threadIdx.x] = 0;
    __syncthreads();
    const int64_t n_nodes = off[P.n];
    int maxl = 0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P.n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int k = off[p + 1] - off[p];
        if (k == 0) continue;
        const int c = cd[p];
        for (int t = 0; t < k; ++t) {
            const int l = c + 1 + t;
            const int64_t id = off[p] + t;
            int64_t e = small_cell_end(P, cd, p, l);
            if (e < 0) e = cell_end(P, keys, p, l);
            const int64_t skip = e < P.n ? (int64_t)off[e] : n_nodes;
            const bool leaf = (t == k - 1);
            link[id] = make_int4((int)skip, (int)p, (int)(e - p), l | (leaf ? 0x100 : 0));
            if (!leaf) {
                ilist[ioff[p] + t] = (int32_t)id;
                atomicAdd(&s_lc[l], 1);
            } else {
                leaves[off[p] - ioff[p]] = (int32_t)id;   // leaves before p = nodes - inner nodes before p
            }
            maxl = l > maxl ? l : maxl;
        }
    }
    __syncthreads();
    if (threadIdx.x <= AG_MAX_LEVEL && s_lc[threadIdx.x] > 0)
        atomicAdd(reinterpret_cast<int32_t*>(hdr + 8) + kLvlCnt + threadIdx.x, s_lc[threadIdx.x]);
    // per-block deepest level (reduced by k_tree_close, no global atomics)
    __shared__ int s_max[kThreads / 64];
    maxl = ag_wave_max(maxl);
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = maxl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int mb = s_max[0];
        for (int w = 1; w < kThreads / 64; ++w) mb = s_max[w] > mb ? s_max[w] : mb;
        blk_max[blockIdx.x] = mb;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        hdr[0] = n_nodes;
        hdr[2] = ioff[P.n];   // inner nodes
    }
}

// One block closes the topology: hdr[1] = deepest level (from the per-block
// maxima of k_write_nodes) and the root node of every system.
__global__ void k_tree_close(int nblk, const int32_t* __restrict__ blk_max, int64_t* __restrict__ hdr, int n_sys,
                             int sys_levels, const int64_t* __restrict__ off, const int32_t* __restrict__ cd,
                             const int32_t* __restrict__ noff, int32_t* __restrict__ root) {
    int m = 0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) m = blk_max[b] > m ? blk_max[b] : m;
    m = ag_wave_max(m);
    __shared__ int s_m[16];
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = s_m[w] > m ? s_m[w] : m;
        m = s_m[0] > m ? s_m[0] : m;
        hdr[1] = m;
    }
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

// lo4.w holds the largest softening length in the node (0 without
// per-particle softening)
__device__ void store_node(int64_t id, const double* r, double4* __restrict__ com, float4* __restrict__ lo4,
                           float4* __restrict__ hi4, float4* __restrict__ mp, double* __restrict__ m64,
                           float hmax) {
    double* o = m64 + id * kM64;
#pragma unroll
    for (int k = 0; k < kM64; ++k) o[k] = r[k];
    double L = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double e = r[22 + c] - r[19 + c];
        L = e > L ? e : L;
    }
    com[id] = make_double4(r[1], r[2], r[3], L);
    lo4[id] = make_float4(f_down(r[19]), f_down(r[20]), f_down(r[21]), hmax);
    hi4[id] = make_float4(f_up(r[22]), f_up(r[23]), f_up(r[24]), (float)r[0]);   // w: mass
    float4* q = mp + 4 * id;
    q[0] = make_float4((float)r[0], (float)r[4], (float)r[5], (float)r[6]);
    q[1] = make_float4((float)r[7], (float)r[8], (float)r[9], (float)r[10]);
    q[2] = make_float4((float)r[11], (float)r[12], (float)r[13], (float)r[14]);
    q[3] = make_float4((float)r[15], (float)r[16], (float)r[17], (float)r[18]);
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
        const double Mi = M > 0.0 ? 1.0 / M : 0.0;
        double E[3] = {0, 0, 0}, F[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c) {
            r[19 + c] = lo[c];
            r[22 + c] = hi[c];
        }
        if (M > 0.0) {
            for (int c = 0; c < 3; ++c) {
                E[c] = e[c] * Mi;
                F[c] = f[c] * Mi;
                r[1 + c] = r0[c] + E[c];
                r[4 + c] = u0[c] + F[c];
            }
        } else {   // massless cell: centre of its box, velocity zero
            for (int c = 0; c < 3; ++c) {
                r[1 + c] = 0.5 * (lo[c] + hi[c]);
                r[4 + c] = 0.0;
            }
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

struct NodeOut {
    double4* com;
    float4* lo4;
    float4* hi4;
    float4* mp;
    double* m64;
    const float* sh;   // sorted softening lengths, or null
};

// sums over the eight lanes of one inner node (one lane per octant)
__device__ __forceinline__ double oct_sum(double v) {
    v += __shfl_xor(v, 1, 8);
    v += __shfl_xor(v, 2, 8);
    v += __shfl_xor(v, 4, 8);
    return v;
}
__device__ __forceinline__ double oct_min(double v) {
    v = fmin(v, __shfl_xor(v, 1, 8));
    v = fmin(v, __shfl_xor(v, 2, 8));
    v = fmin(v, __shfl_xor(v, 4, 8));
    return v;
}
__device__ __forceinline__ double oct_max(double v) {
    v = fmax(v, __shfl_xor(v, 1, 8));
    v = fmax(v, __shfl_xor(v, 2, 8));
    v = fmax(v, __shfl_xor(v, 4, 8));
    return v;
}
__device__ __forceinline__ void oct_reduce(MomentSums& S) {
    S.M = oct_sum(S.M);
    for (int c = 0; c < 3; ++c) {
        S.e[c] = oct_sum(S.e[c]);
        S.f[c] = oct_sum(S.f[c]);
        S.lo[c] = oct_min(S.lo[c]);
        S.hi[c] = oct_max(S.hi[c]);
    }
    for (int k = 0; k < 6; ++k) {
        S.Q[k] = oct_sum(S.Q[k]);
        S.Qd[k] = oct_sum(S.Qd[k]);
    }
}

// every leaf from its particles (one thread per leaf of the dense leaf list;
// a leaf's particles are contiguous and its record is written by one lane,
// which keeps the scattered node writes to one instruction per field)
__global__ void k_leaf_moments(const int64_t* __restrict__ hdr, const int32_t* __restrict__ leaves,
                               const int4* __restrict__ link, const double4* __restrict__ spos,
                               const double4* __restrict__ svel, NodeOut O) {
    const int64_t nl = hdr[0] - hdr[2];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nl;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int id = leaves[t];
        const int4 L = link[id];
        MomentSums S;
        S.init();
        float hm = 0.f;
        for (int q = L.y; q < L.y + L.z; ++q) {
            const double4 a = spos[q];
            const double4 u = svel[q];
            const double x[3] = {a.x, a.y, a.z}, v[3] = {u.x, u.y, u.z};
            S.add(a.w, x, v);
            S.box(x, x);
            if (O.sh) hm = fmaxf(hm, O.sh[q]);
        }
        double r[kM64];
        S.finish(r);
        store_node(id, r, O.com, O.lo4, O.hi4, O.mp, O.m64, hm);
    }
}

// For every inner node: its children by octant (-1 where an octant is
// empty), from the pre-order links (the first child follows the node, the
// next follows the first child's subtree, ...), and its place in the list of
// inner-node indices grouped by level (order within a level is immaterial:
// every block ranks its nodes per level in LDS and takes one slot range per
// level with a global atomic; block 0 also writes the level offsets).
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
        int id = -1, l = 0, r = 0;
        if (t < ni) {
            const int node = ilist[t];
            const int4 L = link[node];
            l = L.w & 0xff;
            id = (int)t;   // listed by inner index
            r = atomicAdd(&s_cnt[l], 1);
            const int sh = 63 - 3 * (l + 1);   // the children's own octal digit
            int c8[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
            for (int ch = node + 1, k8 = 0; ch < L.x && k8 < 8; ++k8) {
                const int4 C = link[ch];
                c8[(int)((keys[C.y] >> sh) & 7)] = ch;
                ch = C.x;
            }
            child[2 * t] = make_int4(c8[0], c8[1], c8[2], c8[3]);
            child[2 * t + 1] = make_int4(c8[4], c8[5], c8[6], c8[7]);
        }
        __syncthreads();
        if (threadIdx.x <= AG_MAX_LEVEL && s_cnt[threadIdx.x] > 0) {
            s_base[threadIdx.x] = atomicAdd(&lvl[kLvlCur + threadIdx.x], s_cnt[threadIdx.x]);
            s_cnt[threadIdx.x] = 0;
        }
        __syncthreads();
        if (id >= 0) lvl_list[s_off[l] + s_base[l] + r] = id;
        __syncthreads();
    }
}

// inner nodes of one level from their children (one launch per level, from
// the deepest up, so every child is complete when its parent is combined).
// Eight lanes per node, one per octant: each lane forms its child's terms
// about the first child's centre of mass and velocity, and the eight lanes
// sum them by shuffles.
__global__ void __launch_bounds__(kThreads) k_inner_level(int level, const int32_t* __restrict__ lvl,
                                                          const int32_t* __restrict__ lvl_list,
                                                          const int32_t* __restrict__ ilist,
                                                          const int32_t* __restrict__ child, NodeOut O) {
    const int t_lo = lvl[kLvlOff + level], t_hi = lvl[kLvlOff + level + 1];
    const int oct = threadIdx.x & 7;
    const int64_t slot = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int64_t nslot = ((int64_t)gridDim.x * blockDim.x) >> 3;
    for (int64_t t = t_lo + slot; t < t_hi; t += nslot) {   // uniform over the eight lanes
        const int in = lvl_list[t];
        const int id = ilist[in];
        const int ch = child[8 * (int64_t)in + oct];
        // the first octant that holds a child supplies the reference point
        const uint64_t occ = __ballot(ch >= 0);
        const unsigned gm = (unsigned)((occ >> (ag_lane() & ~7)) & 0xffu);   // every inner node has a child
        const int chf = gm ? child[8 * (int64_t)in + __builtin_ctz(gm)] : -1;
        MomentSums S;
        S.init();
        for (int c = 0; c < 3; ++c) {
            S.r0[c] = chf >= 0 ? O.m64[(int64_t)chf * kM64 + 1 + c] : 0.0;
            S.u0[c] = chf >= 0 ? O.m64[(int64_t)chf * kM64 + 4 + c] : 0.0;
        }
        S.first = false;
        if (ch >= 0) {
            const double* cm = O.m64 + (int64_t)ch * kM64;
            S.add(cm[0], cm + 1, cm + 4);
            for (int k = 0; k < 6; ++k) {
                S.Q[k] += cm[7 + k];
                S.Qd[k] += cm[13 + k];
            }
            S.box(cm + 19, cm + 22);
        }
        oct_reduce(S);
        float hm = ch >= 0 ? O.lo4[ch].w : 0.f;
        hm = fmaxf(hm, __shfl_xor(hm, 1, 8));
        hm = fmaxf(hm, __shfl_xor(hm, 2, 8));
        hm = fmaxf(hm, __shfl_xor(hm, 4, 8));
        if (oct == 0) {
            double r[kM64];
            S.finish(r);
            store_node(id, r, O.com, O.lo4, O.hi4, O.mp, O.m64, hm);
        }
    }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
int grid_for(int64_t n, int threads = kThreads) {
    int64_t b = (n + threads - 1) / threads;
    if (b > 8192) b = 8192;
    return (int)(b < 1 ? 1 : b);
}

int moments_pass(ag_ctx* c) {
    hipStream_t st = c->stream;
    NodeOut O{c->nd_com.as<double4>(), c->nd_lo.as<float4>(), c->nd_hi.as<float4>(), c->nd_mp.as<float4>(),
              c->nd_64.as<double>(), c->tree_soft ? c->soft_s.as<float>() : nullptr};
    const int64_t n = c->n;
    hipLaunchKernelGGL(k_leaf_moments, dim3(grid_for(n / 4 + 1)), dim3(kThreads), 0, st, c->tree_hdr.as<int64_t>(),
                       c->leaf_list.as<int32_t>(), c->nd_link.as<int4>(), c->spos.as<double4>(),
                       c->svel.as<double4>(), O);
    // level-21 cells are always leaves; empty levels exit at once
    const int64_t inner_bound = c->max_nodes - n;
    int g = grid_for(8 * (inner_bound > 0 ? inner_bound : 1));
    if (g > 1024) g = 1024;
    const int32_t* lvl = reinterpret_cast<const int32_t*>(c->tree_hdr.as<int64_t>() + 8);
    for (int l = AG_MAX_LEVEL - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_inner_level, dim3(g), dim3(kThreads), 0, st, l, lvl, c->lvl_list.as<int32_t>(),
                           c->in_list.as<int32_t>(), c->child.as<int32_t>(), O);
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
    AG_TRY(ag_ensure(c, c->sort_hist, (size_t)(256 * nblocks + 256 + 1) * 4));
    AG_TRY(ag_ensure(c, c->pos_off, (size_t)(256 * (int64_t)nblocks + 1 > n + 1 ? 256 * (int64_t)nblocks + 1 : n + 1) * 4));
    AG_TRY(ag_ensure(c, c->perm, n * 4)); AG_TRY(ag_ensure(c, c->rank, n * 4));
    AG_TRY(ag_ensure(c, c->spos, n * 32)); AG_TRY(ag_ensure(c, c->svel, n * 32)); AG_TRY(ag_ensure(c, c->svf, n * 16));
    AG_TRY(ag_ensure(c, c->cdig, n * 4)); AG_TRY(ag_ensure(c, c->pos_cnt, (n + 1) * 4));
    AG_TRY(ag_ensure(c, c->nd_com, max_nodes * 32)); AG_TRY(ag_ensure(c, c->nd_lo, max_nodes * 16));
    AG_TRY(ag_ensure(c, c->nd_hi, max_nodes * 16)); AG_TRY(ag_ensure(c, c->nd_link, max_nodes * 16));
    AG_TRY(ag_ensure(c, c->nd_mp, max_nodes * 64)); AG_TRY(ag_ensure(c, c->nd_64, max_nodes * kM64 * 8));
    AG_TRY(ag_ensure(c, c->in_list, max_nodes * 4)); AG_TRY(ag_ensure(c, c->in_cnt, (n + 1) * 4));
    AG_TRY(ag_ensure(c, c->in_off, (n + 1) * 4));
    AG_TRY(ag_ensure(c, c->sys_off, (n_sys + 1) * 8)); AG_TRY(ag_ensure(c, c->sys_root, (n_sys + 1) * 4));
    const int64_t inner_bound = max_nodes - n;   // inner nodes never exceed this
    AG_TRY(ag_ensure(c, c->lvl_list, (size_t)(inner_bound > 0 ? inner_bound : 1) * 4));
    AG_TRY(ag_ensure(c, c->leaf_list, n * 4));   // at most one leaf starts at each position
    AG_TRY(ag_ensure(c, c->child, (size_t)(inner_bound > 0 ? inner_bound : 1) * 32));
    AG_TRY(ag_ensure(c, c->sys_box, 6 * n_sys * 8 + 8 * (n_sys + 1)));

    PhaseScope phase(c, AG_PHASE_BUILD);
    hipStream_t st = c->stream;
    int32_t* flags = c->dflags.as<int32_t>();
    int64_t* off = c->sys_off.as<int64_t>();
    int64_t* hdr = c->tree_hdr.as<int64_t>();

    // 1. bounding cubes
    uint64_t* box = c->sys_box.as<uint64_t>();
    int32_t* blk_off = reinterpret_cast<int32_t*>(box + 6 * n_sys);
    hipLaunchKernelGGL(k_build_init, dim3(1), dim3(512), 0, st, n_sys, n, sys_offsets, off, flags, box, blk_off, hdr,
                       (int)(kTreeHdrBytes / 8));
    const int64_t box_blocks = n / kBoxChunk + n_sys + 1;
    hipLaunchKernelGGL(k_box, dim3((unsigned)box_blocks), dim3(kThreads), 0, st, x, off, n_sys, blk_off, box, flags,
                       c->box);

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
    hipLaunchKernelGGL(k_to_sorted, dim3(grid_for(n)), dim3(kThreads), 0, st, n, rank, x, v, m,
                       c->spos.as<double4>(), c->svel.as<double4>(), c->svf.as<float4>(), c->box,
                       c->tree_soft ? c->soft_h.as<double>() : nullptr, c->soft_s.as<float>());
    c->tree_box = c->box;

    // 5. topology
    int32_t* cd = c->cdig.as<int32_t>();
    hipLaunchKernelGGL(k_cdig, dim3(grid_for(n)), dim3(kThreads), 0, st, n, k0, cd);
    TopoParams P{n, n_leaf, sys_levels};
    int32_t* pcnt = c->pos_cnt.as<int32_t>();
    int32_t* poff = c->pos_off.as<int32_t>();
    int32_t* icnt = c->in_cnt.as<int32_t>();
    int32_t* ioff = c->in_off.as<int32_t>();
    hipLaunchKernelGGL(k_count_nodes, dim3(grid_for(n)), dim3(kThreads), 0, st, P, cd, pcnt, icnt);
    AG_TRY(ag_scan_i32(c, pcnt, poff, n));
    AG_TRY(ag_scan_i32(c, icnt, ioff, n));
    const int wblocks = grid_for(n);
    int32_t* blk_max = c->sort_hist.as<int32_t>();   // free after the sort; >= 256 nblocks entries
    hipLaunchKernelGGL(k_write_nodes, dim3(wblocks), dim3(kThreads), 0, st, P, k0, cd, poff, ioff,
                       c->nd_link.as<int4>(), c->in_list.as<int32_t>(), c->leaf_list.as<int32_t>(), hdr, blk_max);
    hipLaunchKernelGGL(k_tree_close, dim3(1), dim3(1024), 0, st, wblocks, blk_max, hdr, n_sys, sys_levels, off, cd,
                       poff, c->sys_root.as<int32_t>());
    hipLaunchKernelGGL(k_level_lists, dim3(grid_for(inner_bound) < 1024 ? grid_for(inner_bound) : 1024),
                       dim3(kThreads), 0, st, hdr, c->in_list.as<int32_t>(), c->nd_link.as<int4>(), k0,
                       c->child.as<int4>(), reinterpret_cast<int32_t*>(hdr + 8), c->lvl_list.as<int32_t>());

    c->n = n;
    c->n_leaf = n_leaf;
    c->n_sys = n_sys;
    c->sys_levels = sys_levels;
    c->max_nodes = max_nodes;

    // 6. moments
    return moments_pass(c);
}

int ag_launch_refit(ag_ctx* c, const double* x, const double* v, const double* m) {
    const int64_t n = c->n;
    PhaseScope phase(c, AG_PHASE_BUILD);
    hipLaunchKernelGGL(k_to_sorted, dim3(grid_for(n)), dim3(kThreads), 0, c->stream, n, c->rank.as<int32_t>(), x,
                       v, m, c->spos.as<double4>(), c->svel.as<double4>(), c->svf.as<float4>(), c->tree_box,
                       c->tree_soft ? c->soft_h.as<double>() : nullptr, c->soft_s.as<float>());
    return moments_pass(c);
}
