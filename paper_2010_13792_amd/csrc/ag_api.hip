// ag_api.hip -- the C ABI entry points: argument validation, context and
// buffer management, dispatch to the kernel launchers.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "ag_internal.h"

static thread_local char g_err[512] = "";

int ag_fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

extern "C" const char* ag_last_error(void) { return g_err; }

int ag_ensure(ag_ctx* c, DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return AG_OK;
    // a captured graph holds the buffers' addresses: none may move while
    // capturing, and a later move invalidates the graph (see ag_graph_replay)
    if (c->capturing)
        return ag_fail(AG_ESTATE, "a library buffer must grow to %zu bytes during graph capture: run the same "
                       "sequence once before capturing", bytes);
    if (c->mem_limit > 0 && c->dev_bytes - b.bytes + bytes > c->mem_limit)
        return ag_fail(AG_ENOMEM, "growing a buffer to %zu bytes would take the context's buffers to %zu bytes, "
                       "past its memory limit of %zu", bytes, c->dev_bytes - b.bytes + bytes, c->mem_limit);
    ++c->alloc_epoch;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        c->dev_bytes -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess) return ag_fail(AG_EHIP, "hipFree failed: %s", hipGetErrorString(e));
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return ag_fail(AG_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    b.bytes = bytes;
    c->dev_bytes += bytes;
    return AG_OK;
}

void ag_release(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

static hipEvent_t take_event(Timing& t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

PhaseScope::PhaseScope(ag_ctx* ctx, int ph) : c(ctx), phase(ph) {
    if (!c->timing.on || ph < 0) return;   // a negative phase records nothing
    a = take_event(c->timing);
    if (a) (void)hipEventRecord(a, c->stream);
}

PhaseScope::~PhaseScope() {
    if (!a) return;
    hipEvent_t b = take_event(c->timing);
    if (!b) {
        c->timing.pool.push_back(a);
        return;
    }
    (void)hipEventRecord(b, c->stream);
    c->timing.pending.push_back({phase, a, b});
}

extern "C" int ag_timing_enable(ag_ctx* c, int enable) {
    if (!c) return ag_fail(AG_EINVAL, "null context");
    c->timing.on = enable != 0;
    return AG_OK;
}

extern "C" int ag_timing_read(ag_ctx* c, double* ms, int64_t* launches, int reset) {
    if (!c) return ag_fail(AG_EINVAL, "null context");
    if (!ms) return ag_fail(AG_EINVAL, "ms is null");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != c->device) (void)hipSetDevice(c->device);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) {
        for (PhaseEvents& p : c->timing.pending) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
                c->timing.ms[p.phase] += t;
                c->timing.launches[p.phase] += 1;
            }
            c->timing.pool.push_back(p.a);
            c->timing.pool.push_back(p.b);
        }
        c->timing.pending.clear();
    }
    for (int k = 0; k < AG_NPHASE; ++k) {
        ms[k] = c->timing.ms[k];
        if (launches) launches[k] = c->timing.launches[k];
        if (reset) {
            c->timing.ms[k] = 0.0;
            c->timing.launches[k] = 0;
        }
    }
    if (prev >= 0 && prev != c->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return ag_fail(AG_EHIP, "stream synchronize failed: %s", hipGetErrorString(e));
    return AG_OK;
}

namespace {

int check_ctx(ag_ctx* c) {
    if (!c) return ag_fail(AG_EINVAL, "null context");
    return AG_OK;
}

int check_launch(const char* what) { return ag_check_launch(what); }

int read_flags(ag_ctx* c) {
    int32_t f = 0;
    AG_HIP(hipMemcpyAsync(&f, c->dflags.p, sizeof(f), hipMemcpyDeviceToHost, c->stream));
    AG_HIP(hipStreamSynchronize(c->stream));
    if (f) {
        AG_HIP(hipMemsetAsync(c->dflags.p, 0, sizeof(int32_t), c->stream));
        AG_HIP(hipStreamSynchronize(c->stream));
        if (f & AGF_NONFINITE) return ag_fail(AG_ENONFINITE, "non-finite particle position in tree build");
        if (f & AGF_INTERNAL) return ag_fail(AG_EHIP, "internal consistency check failed in a tree kernel");
        return ag_fail(AG_EDEVICE, "index list held an out-of-range or repeated entry");
    }
    return AG_OK;
}

}  // namespace

int ag_check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ag_fail(AG_EHIP, "%s: kernel launch failed: %s", what, hipGetErrorString(e));
    return AG_OK;
}

extern "C" int ag_create(ag_ctx** out, int device, void* stream) {
    if (!out) return ag_fail(AG_EINVAL, "out is null");
    *out = nullptr;
    int ndev = 0;
    AG_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return ag_fail(AG_EINVAL, "device %d out of range (%d devices)", device, ndev);
    ag_ctx* c = new (std::nothrow) ag_ctx();
    if (!c) return ag_fail(AG_ENOMEM, "host allocation failed");
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    DeviceGuard g(device);
    int r = ag_direct_noalloc_init(device);
    if (r != AG_OK) {
        delete c;
        return r;
    }
    r = ag_ensure(c, c->stats, 4 * sizeof(uint64_t));
    if (r == AG_OK) r = ag_ensure(c, c->dflags, 4 * sizeof(int32_t));
    if (r == AG_OK) r = ag_ensure(c, c->tree_hdr, kTreeHdrBytes);
    if (r != AG_OK) {
        ag_destroy(c);
        return r;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&c->depth_host), sizeof(int64_t), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->depth_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        ag_destroy(c);
        return ag_fail(AG_EHIP, "context initialisation failed (pinned depth word)");
    }
    if (hipMemsetAsync(c->stats.p, 0, 4 * sizeof(uint64_t), c->stream) != hipSuccess ||
        hipMemsetAsync(c->dflags.p, 0, 4 * sizeof(int32_t), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        ag_destroy(c);
        return ag_fail(AG_EHIP, "context initialisation failed");
    }
    *out = c;
    return AG_OK;
}

extern "C" int ag_destroy(ag_ctx* c) {
    if (!c) return AG_OK;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    DevBuf* bufs[] = {&c->keys[0], &c->keys[1], &c->vals[0], &c->vals[1], &c->sort_hist, &c->perm,
                      &c->rank, &c->spos, &c->svf, &c->cdig, &c->cd_min, &c->pos_cnt, &c->pos_off,
                      &c->scan_tmp, &c->nd_com, &c->nd_lo, &c->nd_hi, &c->nd_link, &c->nd_mp,
                      &c->nd_64, &c->nd_w, &c->nd_wf, &c->in_list, &c->in_cnt, &c->in_off,
                      &c->tree_hdr, &c->lvl_list, &c->leaf_list, &c->leaf_pos, &c->child, &c->sys_off, &c->sys_root, &c->sys_box, &c->act_flag,
                      &c->act_pos, &c->act_off, &c->grp, &c->grp_hdr, &c->ewald_tab, &c->ewald_q, &c->soft_h, &c->soft_s, &c->rel_a, &c->pm_brk, &c->grp_cnt, &c->grp_off, &c->sys_act, &c->wsorted,
                      &c->direct_part, &c->tmp_tidal, &c->sel_flag, &c->sel_off, &c->stats, &c->dflags};
    for (DevBuf* b : bufs) ag_release(*b);
    for (PhaseEvents& p : c->timing.pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (hipEvent_t e : c->timing.pool) (void)hipEventDestroy(e);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->depth_ev) (void)hipEventDestroy(c->depth_ev);
    if (c->depth_host) (void)hipHostFree(c->depth_host);
    delete c;
    return AG_OK;
}

extern "C" int ag_set_stream(ag_ctx* c, void* stream) {
    AG_TRY(check_ctx(c));
    c->stream = reinterpret_cast<hipStream_t>(stream);
    return AG_OK;
}

extern "C" int ag_sync(ag_ctx* c) {
    AG_TRY(check_ctx(c));
    DeviceGuard g(c->device);
    AG_HIP(hipStreamSynchronize(c->stream));
    return read_flags(c);
}

extern "C" int ag_stats_reset(ag_ctx* c) {
    AG_TRY(check_ctx(c));
    DeviceGuard g(c->device);
    AG_HIP(hipMemsetAsync(c->stats.p, 0, 4 * sizeof(uint64_t), c->stream));
    return AG_OK;
}

extern "C" int ag_stats_read(ag_ctx* c, ag_stats* out) {
    AG_TRY(check_ctx(c));
    if (!out) return ag_fail(AG_EINVAL, "out is null");
    DeviceGuard g(c->device);
    uint64_t s[4] = {0, 0, 0, 0};
    int64_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    AG_HIP(hipMemcpyAsync(s, c->stats.p, sizeof(s), hipMemcpyDeviceToHost, c->stream));
    AG_HIP(hipMemcpyAsync(h, c->tree_hdr.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    AG_HIP(hipStreamSynchronize(c->stream));
    out->n_pp = s[0];
    out->n_pn = s[1];
    out->n_targets = s[2];
    out->n_nodes = c->built ? h[0] : 0;
    out->n_leaf = c->built ? c->n_leaf : 0;
    out->max_level = c->built ? (int32_t)h[1] : 0;
    out->n_groups = s[3];
    return read_flags(c);
}

// ---------------------------------------------------------------------------
// tree
// ---------------------------------------------------------------------------
static int build_common(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                        int32_t n_sys, const int64_t* offs, int32_t n_leaf, bool batched) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive (got %lld)", (long long)n);
    if (n > (int64_t)1 << 30) return ag_fail(AG_EINVAL, "n = %lld exceeds 2^30", (long long)n);
    if (!x || !v || !m) return ag_fail(AG_EINVAL, "x, v and m must be non-null");
    if (n_leaf < 1 || n_leaf > 64) return ag_fail(AG_EINVAL, "n_leaf must be in [1, 64] (got %d)", n_leaf);
    if (n_sys < 1 || n_sys > AG_MAX_SYS) return ag_fail(AG_EINVAL, "n_sys must be in [1, %d]", AG_MAX_SYS);
    if (batched && !offs) return ag_fail(AG_EINVAL, "sys_offsets must be non-null");
    if (c->soft_n > 0 && c->soft_n != n)
        return ag_fail(AG_ESTATE, "softening lengths were set for %lld particles, not %lld", (long long)c->soft_n,
                       (long long)n);
    DeviceGuard g(c->device);
    c->built = false;
    c->host_n_nodes = -1;
    int r = ag_launch_build(c, n, x, v, m, n_sys, offs, n_leaf);
    if (r != AG_OK) return r;
    AG_TRY(check_launch("tree build"));
    c->built = true;
    c->batched = batched;
    return AG_OK;
}

extern "C" int ag_tree_build(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                             int32_t n_leaf) {
    return build_common(c, n, x, v, m, 1, nullptr, n_leaf, false);
}

extern "C" int ag_tree_build_batched(ag_ctx* c, int64_t n, const double* x, const double* v,
                                     const double* m, int32_t n_sys, const int64_t* offs, int32_t n_leaf) {
    return build_common(c, n, x, v, m, n_sys, offs, n_leaf, true);
}

extern "C" int ag_tree_refit(ag_ctx* c, const double* x, const double* v, const double* m) {
    AG_TRY(check_ctx(c));
    if (!c->built) return ag_fail(AG_ESTATE, "refit before a tree build");
    if (!x || !v || !m) return ag_fail(AG_EINVAL, "x, v and m must be non-null");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_refit(c, x, v, m));
    return check_launch("tree refit");
}

extern "C" int ag_tree_info(ag_ctx* c, int64_t* n_nodes, int32_t* max_level) {
    AG_TRY(check_ctx(c));
    if (!c->built) return ag_fail(AG_ESTATE, "no tree has been built");
    DeviceGuard g(c->device);
    int64_t h[8];
    AG_HIP(hipMemcpyAsync(h, c->tree_hdr.p, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    AG_HIP(hipStreamSynchronize(c->stream));
    c->host_n_nodes = h[0];
    if (n_nodes) *n_nodes = h[0];
    if (max_level) *max_level = (int32_t)h[1];
    return read_flags(c);
}

extern "C" int ag_tree_export(ag_ctx* c, int64_t cap, int32_t* link, double* moments, int32_t* perm) {
    int64_t nn = 0;
    AG_TRY(ag_tree_info(c, &nn, nullptr));
    if ((link || moments) && cap < nn) return ag_fail(AG_EINVAL, "cap %lld < n_nodes %lld", (long long)cap, (long long)nn);
    DeviceGuard g(c->device);
    if (link) AG_HIP(hipMemcpyAsync(link, c->nd_link.p, nn * 16, hipMemcpyDeviceToDevice, c->stream));
    if (moments) AG_HIP(hipMemcpyAsync(moments, c->nd_64.p, nn * 25 * 8, hipMemcpyDeviceToDevice, c->stream));
    if (perm) AG_HIP(hipMemcpyAsync(perm, c->perm.p, c->n * 4, hipMemcpyDeviceToDevice, c->stream));
    return AG_OK;
}

// ---------------------------------------------------------------------------
// evaluation
// ---------------------------------------------------------------------------
static int check_eval_args(ag_ctx* c, const int32_t* idx, int64_t n_act, double theta, double eps,
                           double G) {
    AG_TRY(check_ctx(c));
    if (!c->built) return ag_fail(AG_ESTATE, "gravity evaluation before a tree build");
    if (c->box != c->tree_box) return ag_fail(AG_ESTATE, "the periodic box changed since the tree was built");
    if (!(eps > 0.0) || !std::isfinite(eps)) return ag_fail(AG_EINVAL, "eps must be positive and finite");
    if (!(theta >= 0.0) || !std::isfinite(theta)) return ag_fail(AG_EINVAL, "theta must be >= 0 and finite");
    if (!std::isfinite(G)) return ag_fail(AG_EINVAL, "G must be finite");
    if (n_act < 0 || n_act > c->n) return ag_fail(AG_EINVAL, "n_active out of range");
    if (c->rel_n > 0 && c->rel_n != c->n)
        return ag_fail(AG_ESTATE, "the relative opening test was set for %lld particles, not %lld",
                       (long long)c->rel_n, (long long)c->n);
    if (!idx && n_act != c->n && n_act != 0)
        return ag_fail(AG_EINVAL, "active_idx = NULL requires n_active = n (or 0)");
    return AG_OK;
}

extern "C" int ag_grav_eval(ag_ctx* c, const int32_t* idx, int64_t n_act, double theta, double eps,
                            double G, double* acc, double* jerk, double* tidal) {
    AG_TRY(check_eval_args(c, idx, n_act, theta, eps, G));
    if (c->batched) return ag_fail(AG_ESTATE, "tree was built batched: use ag_grav_eval_batched");
    if (n_act == 0) return AG_OK;
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_eval(c, idx, n_act, theta, eps, G, acc, jerk, tidal));
    return check_launch("grav eval");
}

extern "C" int ag_grav_eval_dev(ag_ctx* c, const int32_t* idx, const int64_t* n_act_dev, double theta,
                                double eps, double G, double* acc, double* jerk, double* tidal, int64_t* n_total) {
    AG_TRY(check_eval_args(c, idx, c ? c->n : 0, theta, eps, G));
    if (c->batched) return ag_fail(AG_ESTATE, "tree was built batched: use ag_grav_eval_batched");
    if (!idx || !n_act_dev) return ag_fail(AG_EINVAL, "active_idx and n_active_dev must be non-null");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_eval(c, idx, c->n, theta, eps, G, acc, jerk, tidal, n_act_dev, n_total));
    return check_launch("grav eval dev");
}

extern "C" int ag_grav_eval_batched(ag_ctx* c, const int32_t* idx, int64_t n_act, double theta,
                                    double eps, double G, double* acc, double* jerk, double* tidal) {
    AG_TRY(check_eval_args(c, idx, n_act, theta, eps, G));
    if (!c->batched) return ag_fail(AG_ESTATE, "tree was not built batched: use ag_grav_eval");
    if (n_act == 0) return AG_OK;
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_eval(c, idx, n_act, theta, eps, G, acc, jerk, tidal));
    return check_launch("grav eval batched");
}

int ag_direct_check(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m, const int32_t* idx,
                    int64_t n_act, double eps, double G, int precision) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (n > (int64_t)1 << 30) return ag_fail(AG_EINVAL, "n exceeds 2^30");
    if (!x || !v || !m) return ag_fail(AG_EINVAL, "x, v and m must be non-null");
    if (!(eps > 0.0) || !std::isfinite(eps)) return ag_fail(AG_EINVAL, "eps must be positive and finite");
    if (!std::isfinite(G)) return ag_fail(AG_EINVAL, "G must be finite");
    if (precision != AG_FP64 && precision != AG_FP32_PAIRS) return ag_fail(AG_EINVAL, "unknown precision %d", precision);
    if (c->ewald) return ag_fail(AG_ESTATE, "direct summation has no Ewald form (use ag_grav_eval with theta = 0)");
    if (c->soft_n > 0 && c->soft_n != n)
        return ag_fail(AG_ESTATE, "softening lengths were set for %lld particles, not %lld", (long long)c->soft_n,
                       (long long)n);
    if (n_act < 0 || n_act > n) return ag_fail(AG_EINVAL, "n_active out of range");
    if (!idx && n_act != n) return ag_fail(AG_EINVAL, "active_idx = NULL requires n_active = n");
    return AG_OK;
}

extern "C" int ag_grav_direct(ag_ctx* c, int64_t n, const double* x, const double* v, const double* m,
                              const int32_t* idx, int64_t n_act, double eps, double G, int precision,
                              double* acc, double* jerk, double* tidal) {
    AG_TRY(ag_direct_check(c, n, x, v, m, idx, n_act, eps, G, precision));
    if (n_act == 0) return AG_OK;
    DeviceGuard g(c->device);
    const size_t bytes = ag_direct_scratch_bytes(n, n_act, precision);
    if (bytes > 0) AG_TRY(ag_ensure(c, c->direct_part, bytes));
    AG_TRY(ag_launch_direct(c, n, x, v, m, idx, n_act, eps, G, precision, acc, jerk, tidal,
                            bytes > 0 ? c->direct_part.p : nullptr));
    return check_launch("grav direct");
}

extern "C" int ag_grav_timestep(ag_ctx* c, int64_t n, const int32_t* idx, int64_t n_idx,
                                const double* tidal, double eta, double dt_max, int32_t k_max,
                                double* dt, int8_t* bin) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (!tidal || !dt || !bin) return ag_fail(AG_EINVAL, "tidal, dt_grav and bin must be non-null");
    if (!(eta > 0.0) || !std::isfinite(eta)) return ag_fail(AG_EINVAL, "eta must be positive and finite");
    if (!(dt_max > 0.0) || !std::isfinite(dt_max)) return ag_fail(AG_EINVAL, "dt_max must be positive and finite");
    if (k_max < 0 || k_max > 62) return ag_fail(AG_EINVAL, "k_max must be in [0, 62]");
    if (n_idx < 0 || n_idx > n) return ag_fail(AG_EINVAL, "n_idx out of range");
    if (!idx && n_idx != n && n_idx != 0) return ag_fail(AG_EINVAL, "idx = NULL needs n_idx = n (all rows)");
    if (n_idx == 0) return AG_OK;
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_timestep(c, n, idx, n_idx, tidal, eta, dt_max, k_max, dt, bin));
    return check_launch("grav timestep");
}

extern "C" int ag_grav_timestep_dev(ag_ctx* c, int64_t n, const int32_t* idx, const int64_t* n_idx_dev,
                                    const double* tidal, double eta, double dt_max, int32_t k_max, double* dt,
                                    int8_t* bin) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (!idx || !n_idx_dev) return ag_fail(AG_EINVAL, "idx and n_idx_dev must be non-null");
    if (!tidal || !dt || !bin) return ag_fail(AG_EINVAL, "tidal, dt_grav and bin must be non-null");
    if (!(eta > 0.0) || !std::isfinite(eta)) return ag_fail(AG_EINVAL, "eta must be positive and finite");
    if (!(dt_max > 0.0) || !std::isfinite(dt_max)) return ag_fail(AG_EINVAL, "dt_max must be positive and finite");
    if (k_max < 0 || k_max > 62) return ag_fail(AG_EINVAL, "k_max must be in [0, 62]");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_timestep(c, n, idx, n, tidal, eta, dt_max, k_max, dt, bin, n_idx_dev));
    return check_launch("grav timestep dev");
}

extern "C" int ag_adaptive_select(ag_ctx* c, int64_t n, int64_t* tf, const int8_t* bin,
                                  int64_t step_ticks, int32_t tick_bin, double q_f, int32_t* active_idx,
                                  int64_t* n_active_dev, double* t0, double t) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (n > (int64_t)1 << 30) return ag_fail(AG_EINVAL, "n exceeds 2^30");
    if (!tf || !bin || !active_idx || !n_active_dev) return ag_fail(AG_EINVAL, "null pointer argument");
    if (step_ticks < 0) return ag_fail(AG_EINVAL, "step_ticks must be >= 0");
    if (tick_bin < 0 || tick_bin > 52) return ag_fail(AG_EINVAL, "tick_bin must be in [0, 52]");
    if (!(q_f >= 0.0) || !std::isfinite(q_f)) return ag_fail(AG_EINVAL, "q_f must be >= 0 and finite");
    if (t0 && !std::isfinite(t)) return ag_fail(AG_EINVAL, "t must be finite");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_select(c, n, tf, bin, step_ticks, tick_bin, q_f, active_idx, n_active_dev, t0, t));
    return check_launch("adaptive select");
}

extern "C" int ag_kick_drift(ag_ctx* c, int64_t n, double* x, double* v, const double* acc, double dt_kick,
                             double dt_drift) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (!x || !v || !acc) return ag_fail(AG_EINVAL, "null pointer argument");
    if (!std::isfinite(dt_kick) || !std::isfinite(dt_drift)) return ag_fail(AG_EINVAL, "non-finite step");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_kick_drift(c, n, x, v, acc, dt_kick, dt_drift));
    return check_launch("kick drift");
}

extern "C" int ag_set_option(ag_ctx* c, int32_t option, int64_t value) {
    AG_TRY(check_ctx(c));
    switch (option) {
        case AG_OPT_WALK_WAVES_PER_CU:
            if (value < 1 || value > 64) return ag_fail(AG_EINVAL, "walk waves per CU must be in [1, 64]");
            c->walk_waves_per_cu = (int)value;
            return AG_OK;
        case AG_OPT_SMALL_NODE:
            if (value < 0 || value > 16) return ag_fail(AG_EINVAL, "small-node size must be in [0, 16]");
            c->small_node = (int)value;
            return AG_OK;
        case AG_OPT_GROUP_SPAN:
            if (value != 0 && (value < 64 || value > ((int64_t)1 << 30)))
                return ag_fail(AG_EINVAL, "group span must be 0 or in [64, 2^30]");
            c->group_span = (int)value;
            return AG_OK;
        case AG_OPT_GROUP_TARGETS:
            if (value < 1 || value > 64) return ag_fail(AG_EINVAL, "targets per group must be in [1, 64]");
            c->group_cap = (int)value;
            return AG_OK;
        case AG_OPT_EWALD_OPEN:
            if (value < 1 || value > 64) return ag_fail(AG_EINVAL, "Ewald opening value must be in [1, 64]");
            c->ewald_open = (int)value;
            return AG_OK;
        case AG_OPT_ADJOINT_OPEN:
            if (value < 10 || value > 100) return ag_fail(AG_EINVAL, "adjoint opening percentage must be in [10, 100]");
            c->adj_open = (int)value;
            return AG_OK;
        case AG_OPT_GROUP_SPLIT:
            if (value != 0 && (value < 33 || value > 64))
                return ag_fail(AG_EINVAL, "group split bound must be 0 or in [33, 64]");
            c->group_split = (int)value;
            return AG_OK;
        case AG_OPT_GROUP_PACK:
            if (value != 0 && value != 1) return ag_fail(AG_EINVAL, "group packing flag must be 0 or 1");
            c->group_pack = (int)value;
            return AG_OK;
        case AG_OPT_MEM_LIMIT:
            if (value < 0) return ag_fail(AG_EINVAL, "memory limit must be >= 0 bytes (0: none)");
            c->mem_limit = (size_t)value;
            return AG_OK;
        case AG_OPT_MAC_OFFSET:
            if (value != 0 && value != 1) return ag_fail(AG_EINVAL, "opening-test offset flag must be 0 or 1");
            c->mac_offset = (int)value;
            return AG_OK;
        default:
            return ag_fail(AG_EINVAL, "unknown option %d", option);
    }
}

// softening lengths that are not positive and finite raise the device flag
__global__ void k_check_soft(int64_t n, const double* __restrict__ h, int32_t* __restrict__ flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!(h[i] > 0.0) || !isfinite(h[i])) atomicOr(flags, AGF_NONFINITE);
}

extern "C" int ag_set_softening(ag_ctx* c, int64_t n, const double* h) {
    AG_TRY(check_ctx(c));
    if (!h || n == 0) {
        c->soft_n = 0;
        return AG_OK;
    }
    if (n < 0 || n > (int64_t)1 << 30) return ag_fail(AG_EINVAL, "n must be in [0, 2^30]");
    DeviceGuard g(c->device);
    AG_TRY(ag_ensure(c, c->soft_h, (size_t)n * sizeof(double)));
    AG_HIP(hipMemcpyAsync(c->soft_h.p, h, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_check_soft, dim3((unsigned)blocks), dim3(256), 0, c->stream, n, c->soft_h.as<double>(),
                       c->dflags.as<int32_t>());
    c->soft_n = n;
    return check_launch("set softening");
}

// |a| of the previous evaluation as FP32, rounded down (the test then opens
// at least as often as with the exact value); non-finite values raise the flag
__global__ void k_rel_norm(int64_t n, const double* __restrict__ acc, float* __restrict__ out,
                           int32_t* __restrict__ flags) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = sqrt(acc[3 * i] * acc[3 * i] + acc[3 * i + 1] * acc[3 * i + 1] + acc[3 * i + 2] * acc[3 * i + 2]);
        if (!isfinite(a)) atomicOr(flags, AGF_NONFINITE);
        float f = (float)a;
        if ((double)f > a) f = nextafterf(f, 0.f);
        out[i] = isfinite(a) ? f : 0.f;
    }
}

extern "C" int ag_set_relative_opening(ag_ctx* c, double alpha, int64_t n, const double* acc) {
    AG_TRY(check_ctx(c));
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return ag_fail(AG_EINVAL, "alpha must be >= 0 and finite");
    if (alpha == 0.0 || !acc || n == 0) {
        c->rel_n = 0;
        return AG_OK;
    }
    if (n < 0 || n > (int64_t)1 << 30) return ag_fail(AG_EINVAL, "n must be in [0, 2^30]");
    DeviceGuard g(c->device);
    AG_TRY(ag_ensure(c, c->rel_a, (size_t)n * sizeof(float)));
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_rel_norm, dim3((unsigned)blocks), dim3(256), 0, c->stream, n, acc, c->rel_a.as<float>(),
                       c->dflags.as<int32_t>());
    c->rel_n = n;
    c->rel_alpha = alpha;
    return check_launch("set relative opening");
}

extern "C" int ag_set_periodic(ag_ctx* c, double box, int32_t ewald) {
    AG_TRY(check_ctx(c));
    if (!(box >= 0.0) || !std::isfinite(box)) return ag_fail(AG_EINVAL, "box must be >= 0 and finite");
    if (ewald != 0 && ewald != 1) return ag_fail(AG_EINVAL, "ewald must be 0 or 1");
    if (ewald && box == 0.0) return ag_fail(AG_EINVAL, "Ewald sums need a periodic box");
    c->box = box;
    c->ewald = ewald;
    return AG_OK;
}

extern "C" int ag_graph_begin(ag_ctx* c) {
    AG_TRY(check_ctx(c));
    if (c->capturing) return ag_fail(AG_ESTATE, "already capturing");
    if (c->stream == nullptr) return ag_fail(AG_ESTATE, "capture needs a non-default stream");
    if (c->timing.on) return ag_fail(AG_ESTATE, "disable timing before capturing");
    DeviceGuard g(c->device);
    AG_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->capturing = true;
    return AG_OK;
}

extern "C" int ag_graph_end(ag_ctx* c) {
    AG_TRY(check_ctx(c));
    if (!c->capturing) return ag_fail(AG_ESTATE, "not capturing");
    DeviceGuard g(c->device);
    c->capturing = false;
    hipGraph_t gr = nullptr;
    AG_HIP(hipStreamEndCapture(c->stream, &gr));
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph = gr;
    c->graph_exec = nullptr;
    AG_HIP(hipGraphInstantiate(&c->graph_exec, gr, nullptr, nullptr, 0));
    c->graph_epoch = c->alloc_epoch;
    return AG_OK;
}

extern "C" int ag_graph_replay(ag_ctx* c) {
    AG_TRY(check_ctx(c));
    if (!c->graph_exec) return ag_fail(AG_ESTATE, "no captured graph");
    if (c->alloc_epoch != c->graph_epoch)
        return ag_fail(AG_ESTATE, "a library buffer was reallocated after the capture (a later call needed more "
                       "scratch): capture the sequence again");
    DeviceGuard g(c->device);
    AG_HIP(hipGraphLaunch(c->graph_exec, c->stream));
    return AG_OK;
}

extern "C" int ag_grav_predict(ag_ctx* c, int64_t n, const uint8_t* mask, const double* a0,
                               const double* j, const double* t0, double t, double* out) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (!a0 || !out || (j && !t0)) return ag_fail(AG_EINVAL, "null pointer argument");
    if (!std::isfinite(t)) return ag_fail(AG_EINVAL, "t must be finite");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_predict(c, n, mask, a0, j, t0, t, out));
    return check_launch("grav predict");
}

extern "C" int ag_grav_predict_age(ag_ctx* c, int64_t n, const uint8_t* mask, const double* a0, const double* j,
                                   const int64_t* age_ticks, double tick, double* out) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (!a0 || !out || (j && !age_ticks)) return ag_fail(AG_EINVAL, "null pointer argument");
    if (!std::isfinite(tick)) return ag_fail(AG_EINVAL, "tick must be finite");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_predict_age(c, n, mask, a0, j, age_ticks, tick, out));
    return check_launch("grav predict age");
}

extern "C" int ag_force_log(ag_ctx* c, int64_t n, const int32_t* idx, int64_t n_idx, int32_t depth,
                            const double* a0, double t, double* ha, double* ht, int32_t* hn) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (n > (int64_t)1 << 30) return ag_fail(AG_EINVAL, "n exceeds 2^30");
    if (depth < 1 || depth > AG_PRED_MAX_DEPTH) return ag_fail(AG_EINVAL, "depth must be in [1, AG_PRED_MAX_DEPTH]");
    if (!a0 || !ha || !ht || !hn) return ag_fail(AG_EINVAL, "null pointer argument");
    if (!std::isfinite(t)) return ag_fail(AG_EINVAL, "t must be finite");
    if (n_idx < 0 || n_idx > n) return ag_fail(AG_EINVAL, "n_idx out of range");
    if (!idx && n_idx != n && n_idx != 0) return ag_fail(AG_EINVAL, "idx = NULL needs n_idx = n (all rows)");
    if (n_idx == 0) return AG_OK;
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_force_log(c, n, idx, n_idx, depth, a0, t, ha, ht, hn));
    return check_launch("force log");
}

extern "C" int ag_force_log_dev(ag_ctx* c, int64_t n, const int32_t* idx, const int64_t* n_idx_dev, int32_t depth,
                                const double* a0, double t, double* ha, double* ht, int32_t* hn) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (n > (int64_t)1 << 30) return ag_fail(AG_EINVAL, "n exceeds 2^30");
    if (depth < 1 || depth > AG_PRED_MAX_DEPTH) return ag_fail(AG_EINVAL, "depth must be in [1, AG_PRED_MAX_DEPTH]");
    if (!idx || !n_idx_dev || !a0 || !ha || !ht || !hn) return ag_fail(AG_EINVAL, "null pointer argument");
    if (!std::isfinite(t)) return ag_fail(AG_EINVAL, "t must be finite");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_force_log(c, n, idx, n, depth, a0, t, ha, ht, hn, n_idx_dev));
    return check_launch("force log dev");
}

extern "C" int ag_grav_predict_poly(ag_ctx* c, int64_t n, const uint8_t* mask, int32_t depth, int32_t order,
                                    const double* ha, const double* ht, const int32_t* hn, double t,
                                    double* out) {
    AG_TRY(check_ctx(c));
    if (n <= 0) return ag_fail(AG_EINVAL, "n must be positive");
    if (n > (int64_t)1 << 30) return ag_fail(AG_EINVAL, "n exceeds 2^30");
    if (depth < 1 || depth > AG_PRED_MAX_DEPTH) return ag_fail(AG_EINVAL, "depth must be in [1, AG_PRED_MAX_DEPTH]");
    if (order < 0 || order >= depth) return ag_fail(AG_EINVAL, "order must be in [0, depth - 1]");
    if (!ha || !ht || !hn || !out) return ag_fail(AG_EINVAL, "null pointer argument");
    if (!std::isfinite(t)) return ag_fail(AG_EINVAL, "t must be finite");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_predict_poly(c, n, mask, depth, order, ha, ht, hn, t, out));
    return check_launch("grav predict poly");
}

extern "C" int ag_grav_backward(ag_ctx* c, const int32_t* idx, int64_t n_act, const double* w,
                                double theta, double eps, double G, double* dLdx, double* dLdm) {
    AG_TRY(check_eval_args(c, idx, n_act, theta, eps, G));
    if (c->batched) return ag_fail(AG_ESTATE, "backward is not available for a batched tree");
    if (c->box > 0.0) return ag_fail(AG_ESTATE, "backward is not available with periodic boundaries");
    if (c->tree_soft) return ag_fail(AG_ESTATE, "backward is not available with per-particle softening");
    if (c->rel_n > 0) return ag_fail(AG_ESTATE, "backward is not available with the relative opening test");
    if (!w || !dLdx || !dLdm) return ag_fail(AG_EINVAL, "w, dLdx and dLdm must be non-null");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_backward(c, idx, n_act, w, theta, eps, G, dLdx, dLdm));
    return check_launch("grav backward");
}

// state shared by the three calls; a null n_ngb skips its range check
static int check_pm(ag_ctx* c, const double* n_ngb, bool lengths) {
    AG_TRY(check_ctx(c));
    if (!c->built) return ag_fail(AG_ESTATE, "Price & Monaghan terms before a tree build");
    if (c->batched) return ag_fail(AG_ESTATE, "Price & Monaghan terms are not available for a batched tree");
    if (c->tree_box > 0.0) return ag_fail(AG_ESTATE, "Price & Monaghan terms need open boundaries");
    if (!lengths && !c->tree_soft)
        return ag_fail(AG_ESTATE, "the tree was built without per-particle softening lengths");
    if (n_ngb && (!(*n_ngb > 32.0 / 3.0) || !(*n_ngb < 32.0 * (double)c->n / 3.0)))
        return ag_fail(AG_EINVAL, "n_ngb must lie in (32/3, 32 n/3)");
    return AG_OK;
}

extern "C" int ag_pm_lengths(ag_ctx* c, double n_ngb, double* h, double* omega) {
    AG_TRY(check_pm(c, &n_ngb, true));
    if (!h || !omega) return ag_fail(AG_EINVAL, "h and omega must be non-null");
    DeviceGuard g(c->device);
    AG_TRY(ag_ensure(c, c->pm_brk, (size_t)c->n * (3 * sizeof(double) + sizeof(int32_t)) + kPmSteps * sizeof(int)));
    // each step counts in a slot of its own (slot 0: the rows the list pass
    // leaves to the sum walk)
    int* cnt = reinterpret_cast<int*>(c->pm_brk.as<double>() + 3 * c->n);
    AG_HIP(hipMemsetAsync(cnt, 0, kPmSteps * sizeof(int), c->stream));
    AG_TRY(ag_launch_pm_lengths(c, n_ngb, h, omega, 0, 0));
    AG_TRY(check_launch("Price & Monaghan lengths"));
    int32_t f = 0, n_left = 0;
    AG_HIP(hipMemcpyAsync(&f, c->dflags.p, sizeof(f), hipMemcpyDeviceToHost, c->stream));
    AG_HIP(hipMemcpyAsync(&n_left, cnt, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    AG_HIP(hipStreamSynchronize(c->stream));
    if ((f & AGF_PMSHORT) && n_left > 0) {
        // Newton steps of the sum walk until no length moves
        AG_HIP(hipMemsetAsync(c->dflags.p, 0, sizeof(int32_t), c->stream));
        int step = 1, moving = 1;
        for (; step < kPmSteps && moving; ++step) {
            AG_TRY(ag_launch_pm_lengths(c, n_ngb, h, omega, step, n_left));
            if (step % 4 == 0 || step == kPmSteps - 1) {
                AG_HIP(hipMemcpyAsync(&moving, cnt + step, sizeof(int), hipMemcpyDeviceToHost, c->stream));
                AG_HIP(hipStreamSynchronize(c->stream));
            }
        }
        AG_TRY(check_launch("Price & Monaghan lengths"));
        if (moving) return ag_fail(AG_EHIP, "Price & Monaghan lengths did not settle");
    }
    return read_flags(c);
}

extern "C" int ag_pm_factors(ag_ctx* c, double n_ngb, double G, const double* omega, double* z) {
    AG_TRY(check_pm(c, &n_ngb, false));
    if (!omega || !z) return ag_fail(AG_EINVAL, "omega and z must be non-null");
    if (!std::isfinite(G)) return ag_fail(AG_EINVAL, "G must be finite");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_pm_sum(c, 0, n_ngb, G, omega, nullptr, z, nullptr));
    return check_launch("Price & Monaghan factors");
}

extern "C" int ag_pm_correct(ag_ctx* c, const double* z, double* acc) {
    AG_TRY(check_pm(c, nullptr, false));
    if (!z || !acc) return ag_fail(AG_EINVAL, "z and acc must be non-null");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_pm_sum(c, 1, 0.0, 0.0, nullptr, z, nullptr, acc));
    return check_launch("Price & Monaghan correction");
}

extern "C" int ag_pm_correct_add(ag_ctx* c, const double* z, const int32_t* idx, const int64_t* n_idx_dev,
                                 double* acc) {
    AG_TRY(check_pm(c, nullptr, false));
    if (!z || !acc) return ag_fail(AG_EINVAL, "z and acc must be non-null");
    if (idx && !n_idx_dev) return ag_fail(AG_EINVAL, "n_idx_dev must be non-null with idx");
    DeviceGuard g(c->device);
    if (idx) AG_TRY(ag_launch_pm_sum(c, 1, 0.0, 0.0, nullptr, z, nullptr, acc, idx, n_idx_dev));
    else AG_TRY(ag_launch_pm_sum(c, 1, 0.0, 0.0, nullptr, z, nullptr, acc, nullptr, nullptr, true));
    return check_launch("Price & Monaghan correction (added)");
}

extern "C" int ag_neighbour_lengths(ag_ctx* c, int32_t k, double scale, double* h) {
    AG_TRY(check_ctx(c));
    if (!c->built) return ag_fail(AG_ESTATE, "neighbour lengths before a tree build");
    if (c->batched) return ag_fail(AG_ESTATE, "neighbour lengths are not available for a batched tree");
    if (k < 1 || k > 64) return ag_fail(AG_EINVAL, "k must be in [1, 64]");
    if ((int64_t)k >= c->n) return ag_fail(AG_EINVAL, "k must be below the number of particles");
    if (!h) return ag_fail(AG_EINVAL, "h must be non-null");
    if (!(scale > 0.0) || !std::isfinite(scale)) return ag_fail(AG_EINVAL, "scale must be positive and finite");
    DeviceGuard g(c->device);
    AG_TRY(ag_launch_knn(c, k, scale, h));
    return check_launch("neighbour lengths");
}
