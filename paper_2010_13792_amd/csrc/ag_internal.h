// ag_internal.h -- context layout and device helpers shared by the library's
// translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <vector>

#include "adaptgrav.h"

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
int ag_fail(int code, const char* fmt, ...);

#define AG_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            return ag_fail(AG_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define AG_TRY(call)              \
    do {                          \
        int r_ = (call);          \
        if (r_ != AG_OK) return r_; \
    } while (0)

// ---------------------------------------------------------------------------
// device buffers owned by the context (grow-only)
// ---------------------------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// device-side flag bits (ag_ctx::dflags)
enum { AGF_BADINDEX = 1, AGF_NONFINITE = 2, AGF_INTERNAL = 4, AGF_PMSHORT = 8 };

constexpr int AG_MAX_LEVEL = 21;   // Morton digits: 21 x 3 bits = 63-bit keys
constexpr int AG_MAX_SYS = 512;    // batched systems: 3 octal digits of prefix
constexpr int AG_GROUP = 64;       // targets per walk group = one wave64

// level table after the eight i64 header words of tree_hdr (as i32): inner
// nodes per level, a scatter cursor per level, and the level offsets into
// lvl_list (AG_MAX_LEVEL + 1 entries)
constexpr int kLvlCnt = 0, kLvlCur = 32, kLvlOff = 64, kLvlWords = 128;
constexpr size_t kTreeHdrBytes = 8 * sizeof(int64_t) + kLvlWords * sizeof(int32_t);

// per-phase event timing (enabled by ag_timing_enable)
struct PhaseEvents {
    int phase;
    hipEvent_t a, b;
};
struct Timing {
    bool on = false;
    std::vector<PhaseEvents> pending;
    std::vector<hipEvent_t> pool;
    double ms[AG_NPHASE] = {0};
    int64_t launches[AG_NPHASE] = {0};
};

struct ag_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Timing timing;
    int walk_waves_per_cu = 16;
    int small_node = 2;
    int group_span = 128;
    int mac_offset = 1;
    double box = 0.0;     // periodic cube side (0: open boundaries)
    int ewald = 0;        // periodic: Ewald sums for g and T
    int ewald_open = 4;   // correction walk: opening angle 1 / ewald_open against the image points
    double ewald_tab_box = 0.0;   // box the Ewald table was built for
    double tree_box = 0.0;        // periodic box the tree was built in (positions wrapped into it)
    int64_t soft_n = 0;           // per-particle softening lengths set for this many particles (0: none)
    int64_t rel_n = 0;            // relative opening test set for this many particles (0: off)
    double rel_alpha = 0.0;
    bool tree_soft = false;       // the current tree carries them
    int group_cap = 64;
    int group_split = 42;  // groups of 33 .. group_split targets are split in two (0: none)
    int group_pack = 0;    // 1: runs of children are cut every group_cap targets
    bool capturing = false;
    uint64_t alloc_epoch = 0;     // bumped by every (re)allocation of a context buffer
    uint64_t graph_epoch = 0;     // alloc_epoch when the graph was captured
    int adj_open = 75;            // adjoint walks open nodes at adj_open % of theta
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;

    // --- tree state ---
    bool built = false;
    bool batched = false;
    int64_t n = 0;
    int32_t n_leaf = 16;
    int32_t n_sys = 1;
    int32_t sys_levels = 0;  // octal digits taken by the system prefix
    int64_t max_nodes = 0;

    DevBuf keys[2], vals[2];      // radix-sort ping-pong (u64 keys, i32 values)
    DevBuf sort_hist;             // per-block digit counts (u32)
    DevBuf perm;                  // i32 [n]: sorted position -> input row
    DevBuf rank;                  // i32 [n]: input row -> sorted position
    DevBuf spos;                  // double4 [n]: sorted x, y, z, m
    DevBuf svf;                   // float4  [n]: sorted vx, vy, vz, m (FP32 copies)
    DevBuf cdig;                  // i32 [n]: octal digits shared with the previous key
    DevBuf cd_min;                // i32: their minima over runs of 16, 256, ... 2^24 positions
    DevBuf pos_cnt, pos_off;      // i32 [n+1]: nodes starting at each position, offsets
    DevBuf scan_tmp;              // scan block partials

    // node arrays, depth-first (pre-order) numbering
    DevBuf nd_com;                // double4: centre of mass x y z, extent L
    DevBuf nd_lo, nd_hi;          // float4: bounding box (rounded outward)
    DevBuf nd_link;               // int4: skip (next node after subtree), start, count, level|leafbit
    DevBuf nd_mp;                 // float4 x4: M ux uy uz | Q xx yy zz xy | Q xz yz, Qd xx yy | Qd zz xy xz yz
    DevBuf nd_64;                 // double [25]: FP64 moments (M, c, u, Q, Qd, lo, hi)
    DevBuf nd_w;                  // double [12]: vector-charge moments W0 (3), W1 (9) for the adjoint
    DevBuf nd_wf;                 // float4 x3: W0, W1 in FP32 for the adjoint walk
    DevBuf in_list;               // i32 [max_nodes]: inner nodes in pre-order
    DevBuf in_cnt, in_off;        // i32 [n+1]: inner nodes starting at each position, offsets
    DevBuf tree_hdr;              // i64 [8]: n_nodes, max_level, inner nodes; then the level table (kLvl*)
    DevBuf lvl_list;              // i32 [inner bound]: inner node ids grouped by level
    DevBuf leaf_list;             // i32 [n]: leaf node ids in pre-order
    DevBuf leaf_pos;              // i32 [n+1]: first position of each leaf, then n
    DevBuf child;                 // i32 [8 x inner bound]: children by octant (-1: none) of the node in the same lvl_list slot

    DevBuf sys_off;               // i64 [n_sys+1]
    DevBuf sys_root;              // i32 [n_sys]: root node per system
    DevBuf sys_box;               // u64 [6 n_sys]: order-preserving encoded min/max

    // --- evaluation scratch ---
    bool all_active = false;      // the last grouping listed every particle (no flag, offset or position arrays)
    DevBuf act_flag;              // i32 [n]
    DevBuf act_pos;               // i32 [n]: active sorted positions, ascending
    DevBuf act_off;               // i32 [n+1]: exclusive scan of act_flag
    DevBuf grp;                   // int4 [max groups]: start, count, system, -
    DevBuf soft_h;                // f64 per-particle softening lengths, input order
    DevBuf soft_s;                // f32 the same in key order (rounded up)
    DevBuf rel_a;                 // f32 |a| of the previous evaluation, input order (rounded down)
    DevBuf pm_brk;                // Price & Monaghan lengths: brackets and current lengths (3 n doubles), step counters, rows left to the sum walk (n)
    DevBuf ewald_tab;             // f32 Ewald correction table (5 float4 per point)
    DevBuf ewald_q;               // i32 [8]: correction walk work-queue counters
    DevBuf grp_hdr;               // i32: [0] number of groups, [8..15] walk work-queue counters
    DevBuf grp_cnt, grp_off;      // i32 [max_nodes (+1)]: groups owned per node, offsets
    DevBuf sys_act;               // i32 [n_sys + 1]
    DevBuf wsorted;               // double4 [n]: adjoint weights in sorted order
    DevBuf direct_part;           // direct sum: FP64 per-split sums of a small target set
    DevBuf tmp_tidal;             // double [n*6]
    DevBuf sel_flag;              // i32 [n]: due flags of the last select
    DevBuf sel_off;               // i32 [n+1]: their exclusive scan

    // --- counters and flags (device) ---
    DevBuf stats;                 // u64 [4]: n_pp, n_pn, n_targets
    DevBuf dflags;                // i32 [1]

    int64_t host_n_nodes = -1;    // cached after a synchronising read
    size_t dev_bytes = 0;         // bytes held by the buffers above
    size_t mem_limit = 0;         // AG_OPT_MEM_LIMIT (0: none)
    // depth of the last tree seen by the host (pinned copy + event, read when
    // the next build starts without waiting): plans the moments' launches
    int64_t* depth_host = nullptr;
    hipEvent_t depth_ev = nullptr;
    bool depth_pending = false;
    int seen_max_level = -1;
};

// grow-only device buffer of the context (AG_ESTATE while capturing a graph)
int ag_ensure(ag_ctx* c, DevBuf& b, size_t bytes);

// makes a device current for a scope and restores the previous one
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// argument checks of ag_grav_direct (shared by its allocation-free variant)
int ag_direct_check(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m, const int32_t* idx,
                    int64_t n_act, double eps, double G, int precision);
// the allocation-free direct sum's scratch on the current device: looked up
// once per device (ag_create calls it with the device current)
int ag_direct_noalloc_init(int device);
int ag_check_launch(const char* what);
void ag_release(DevBuf& b);

// Records a start event on construction and a stop event on destruction on
// the context's stream, when timing is enabled and the phase is not negative.
struct PhaseScope {
    ag_ctx* c;
    int phase;
    hipEvent_t a = nullptr;
    PhaseScope(ag_ctx* ctx, int ph);
    ~PhaseScope();
};

// ---------------------------------------------------------------------------
// launchers implemented in the kernel translation units
// ---------------------------------------------------------------------------
// direct summation; scratch holds ag_direct_scratch_bytes(n, n_act, precision) bytes (the
// per-split sums of a small target set; nothing need be cleared)
int ag_launch_direct(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                     const int32_t* idx, int64_t n_act, double eps, double G, int precision,
                     double* acc, double* jerk, double* tidal, void* scratch, bool timed = true);
size_t ag_direct_scratch_bytes(int64_t n, int64_t n_act, int precision);
int ag_launch_timestep(ag_ctx* c, int64_t n, const int32_t* idx, int64_t n_idx,
                       const double* tidal, double eta, double dt_max, int32_t k_max,
                       double* dt, int8_t* bin, const int64_t* n_dev = nullptr);
int ag_launch_select(ag_ctx* c, int64_t n, int64_t* tf, const int8_t* bin, int64_t step_ticks,
                     int32_t tick_bin, double q_f, int32_t* active_idx, int64_t* n_active_dev,
                     double* t0, double t);
int ag_launch_kick_drift(ag_ctx* c, int64_t n, double* x, double* v, const double* acc, double dt_kick,
                         double dt_drift);
int ag_launch_predict(ag_ctx* c, int64_t n, const uint8_t* mask, const double* a0,
                      const double* j, const double* t0, double t, double* out);
int ag_launch_predict_age(ag_ctx* c, int64_t n, const uint8_t* mask, const double* a0, const double* j,
                          const int64_t* age, double tick, double* out);
int ag_launch_force_log(ag_ctx* c, int64_t n, const int32_t* idx, int64_t n_idx, int32_t depth,
                        const double* a0, double t, double* ha, double* ht, int32_t* hn,
                        const int64_t* n_dev = nullptr);
int ag_launch_predict_poly(ag_ctx* c, int64_t n, const uint8_t* mask, int32_t depth, int32_t order,
                           const double* ha, const double* ht, const int32_t* hn, double t, double* out);
int ag_launch_build(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                    int32_t n_sys, const int64_t* sys_offsets, int32_t n_leaf);
int ag_launch_refit(ag_ctx* c, const double* x, const double* v, const double* m);
int ag_launch_eval(ag_ctx* c, const int32_t* idx, int64_t n_act, double theta, double eps,
                   double G, double* acc, double* jerk, double* tidal, const int64_t* n_dev = nullptr,
                   int64_t* n_total = nullptr);
int ag_launch_knn(ag_ctx* c, int32_t k, double scale, double* h_out);
constexpr int kPmSteps = 257;   // sum walk steps of the lengths (slot 0 unused) and their counters
int ag_launch_pm_lengths(ag_ctx* c, double n_ngb, double* h, double* omega, int step, int64_t n_left);
// mode 0: Z of every particle into z_out; mode 1: the correction, written to
// acc for every row (idx null; added with `add`) or added to acc at rows
// idx[0 .. *n_dev)
int ag_launch_pm_sum(ag_ctx* c, int mode, double n_ngb, double G, const double* omega, const double* z,
                     double* z_out, double* acc, const int32_t* idx = nullptr, const int64_t* n_dev = nullptr,
                     bool add = false);
int ag_launch_backward(ag_ctx* c, const int32_t* idx, int64_t n_act, const double* w,
                       double theta, double eps, double G, double* dLdx, double* dLdm);
// exclusive scan of n int32 counts into out (n+1 entries; out[n] = total) on c->stream
int ag_scan_i32(ag_ctx* c, const int32_t* in, int32_t* out, int64_t n);
// active rows -> ascending sorted positions and walk groups; returns upper bound of groups.
// With n_dev set the list's length is read on the device (n_act is then its
// capacity) and, with n_total set, added to *n_total on the device.
int ag_prepare_groups(ag_ctx* c, const int32_t* idx, int64_t n_act, int64_t* max_groups, const int64_t* n_dev,
                      int64_t* n_total);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
#if defined(__HIPCC__)
__device__ __forceinline__ int ag_lane() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of `mask` in lanes below this one
__device__ __forceinline__ int ag_prefix_count(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <class T> __device__ __forceinline__ T ag_wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <class T> __device__ __forceinline__ T ag_wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o, 64); v = w < v ? w : v; }
    return v;
}
template <class T> __device__ __forceinline__ T ag_wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { T w = __shfl_xor(v, o, 64); v = w > v ? w : v; }
    return v;
}
// inclusive prefix sum over the wave
__device__ __forceinline__ int ag_wave_incl_scan(int v) {
    const int lane = ag_lane();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int w = __shfl_up(v, o, 64);
        if (lane >= o) v += w;
    }
    return v;
}

// order-preserving map of doubles onto uint64 (for atomic min/max)
__device__ __forceinline__ uint64_t ag_ord(double x) {
    uint64_t b = __double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ag_unord(uint64_t u) {
    uint64_t b = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
    return __longlong_as_double(b);
}
#endif
