/*
 * adaptgrav.h -- C ABI of the MI355X (gfx950) gravity library for adaptive
 * force updates (Grudic 2020, "Accelerating self-gravitating hydrodynamics
 * simulations with adaptive force updates").
 *
 * The library evaluates softened self-gravity -- acceleration g, its time
 * derivative (jerk) j and the tidal tensor T -- for a chosen subset of
 * particles, by direct summation or with a Barnes-Hut oct-tree, and provides
 * the bookkeeping the paper builds around the solver: the tidal timestep
 * (Eq. 7), the force-age counter and update test (Eq. 3, Eq. 4) and the jerk
 * predictor (Eq. 6).  Every step runs in hand-written HIP kernels.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Units: the caller passes G; positions, velocities and masses are in any
 *    consistent units.
 *  - Arrays are caller-owned DEVICE memory (hipMalloc or a torch CUDA/HIP
 *    tensor) unless a parameter says "host".  Layouts are row-major:
 *    vectors are (n, 3) doubles (x0 y0 z0 x1 ...), symmetric tensors are
 *    (n, 6) doubles in xx yy zz xy xz yz order, scalars are (n,).
 *  - Index lists (active_idx) are int32 row numbers in [0, n), unique, in any
 *    order.
 *  - Calls are asynchronous and ordered on the context's stream; input
 *    arrays must stay valid and unchanged until the stream reaches the call.
 *    The library never frees or keeps caller pointers.
 *  - Return value: AG_OK or a negative error code; ag_last_error() gives a
 *    message (per thread).  A failing call leaves the context usable.
 *    Invalid device-resident data (indices out of range or repeated,
 *    non-finite positions) cannot be seen by the host without a wait: kernels
 *    skip such entries and raise a device flag that the next ag_sync() or
 *    ag_stats_read() reports as AG_EDEVICE or AG_ENONFINITE.
 *  - A context is bound to one device and one stream and is not
 *    thread-safe; use one context per host thread.
 *
 * Softening: cubic-spline (M4) kernel of compact support h = eps; pairs
 * closer than eps feel the kernel-smoothed force, beyond it Newton's.  The
 * self pair is excluded.
 */
#ifndef ADAPTGRAV_H
#define ADAPTGRAV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ag_ctx ag_ctx;

enum {
    AG_OK = 0,
    AG_EINVAL = -1,      /* bad argument (n <= 0, eps <= 0, theta < 0, null pointer ...) */
    AG_ENOMEM = -2,      /* device allocation failed */
    AG_EHIP = -3,        /* HIP runtime error; message in ag_last_error() */
    AG_ESTATE = -4,      /* call out of order (eval before build, size mismatch) */
    AG_ENONFINITE = -5,  /* a position was NaN or Inf in the last tree build */
    AG_EDEVICE = -6      /* an index list held an out-of-range or repeated entry */
};

enum { AG_FP64 = 0, AG_FP32_PAIRS = 1 };

/* Counters accumulated on the device since the last ag_stats_reset(). */
typedef struct ag_stats {
    uint64_t n_pp;       /* particle-particle interactions evaluated          */
    uint64_t n_pn;       /* particle-node (multipole) interactions evaluated  */
    uint64_t n_targets;  /* force evaluations: targets given fresh g, j, T    */
    int64_t  n_nodes;    /* nodes of the current tree                          */
    int32_t  n_leaf;     /* leaf capacity of the current tree                  */
    int32_t  max_level;  /* deepest tree level in use                          */
    uint64_t n_groups;   /* target groups walked (one wave each)               */
} ag_stats;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`, bound to the HIP stream `stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the handle. */
int ag_create(ag_ctx **out, int device, void *stream);
/* Release the context and all library-owned device memory (waits for the
 * stream first).  NULL is accepted. */
int ag_destroy(ag_ctx *ctx);
/* Rebind the context to another stream of the same device. */
int ag_set_stream(ag_ctx *ctx, void *stream);
/* Wait for the stream; return AG_OK or the first device-side error raised
 * since the last check (the flag is then cleared). */
int ag_sync(ag_ctx *ctx);
/* Synchronising read of the counters (also reports device errors as ag_sync). */
int ag_stats_read(ag_ctx *ctx, ag_stats *out);
int ag_stats_reset(ag_ctx *ctx);
/* Message for the last failing call on this host thread. */
const char *ag_last_error(void);

/* Tunable launch options (picked by an autotuner; defaults in brackets):
 *   AG_OPT_WALK_WAVES_PER_CU   resident walk waves launched per CU [16]
 *   AG_OPT_SMALL_NODE          accepted nodes with at most this many particles
 *                              are summed pair by pair instead [2]
 *   AG_OPT_GROUP_SPAN          a target group never spans a cell holding more
 *                              than this many particles (active or not), so
 *                              sparse active sets still give compact groups;
 *                              0 = no limit [128]
 *   AG_OPT_MAC_OFFSET          1: the opening test adds the distance from a
 *                              node's centre of mass to the centre of its box
 *                              to the node's extent (opens lopsided nodes
 *                              sooner); 0: extent alone (fewer interactions,
 *                              larger errors) [1]
 *   AG_OPT_GROUP_TARGETS       most targets in one walk group (one wave walks
 *                              the tree per group; a group of k targets gives
 *                              each target min(32, 64 / k) lanes) [64]
 *   AG_OPT_EWALD_OPEN          Ewald correction walk: a node acts as a point
 *                              (mass and quadrupole) if its extent is at most
 *                              1 / value times its distance to the nearest
 *                              image point of the lattice [4]
 *   AG_OPT_ADJOINT_OPEN        ag_grav_backward opens nodes at value % of its
 *                              theta, in both of its walks: their kernels (the
 *                              tidal tensor and J, 1/r^3) are one derivative
 *                              deeper than the force's, and at 75 % they meet
 *                              the force's error bound at the caller's theta [75]
 *   AG_OPT_GROUP_SPLIT         a group of 33 .. value targets is walked as two
 *                              halves (a wave gives each of k targets 64 / k
 *                              whole lanes, so 33 .. 42 targets leave lanes
 *                              idle that halves of 17 .. 21 use); 0 = never [42]
 *   AG_OPT_GROUP_PACK          1: the targets of consecutive child cells (one
 *                              run, inside their parent's cell) are cut into
 *                              groups of AG_OPT_GROUP_TARGETS and a remainder,
 *                              a child's targets possibly in two groups; 0:
 *                              runs are cut between children, so no group
 *                              reaches the cap unless its children fill it [0]
 *   AG_OPT_MEM_LIMIT           most bytes of device memory the context's own
 *                              buffers may hold together; a call that would
 *                              grow them past it fails with AG_ENOMEM before
 *                              freeing or launching anything (a failed build
 *                              leaves no tree: later calls that need one give
 *                              AG_ESTATE until a build succeeds); 0 = no limit
 *                              beyond the device's own [0]
 * Values outside the documented ranges (1..64, 0..16, 0 or 64..2^30, 0..1,
 * 1..64, 1..64, 10..100, 0 or 33..64, 0..1, >= 0) give AG_EINVAL. */
enum { AG_OPT_WALK_WAVES_PER_CU = 1, AG_OPT_SMALL_NODE = 2, AG_OPT_GROUP_SPAN = 3, AG_OPT_MAC_OFFSET = 4,
       AG_OPT_GROUP_TARGETS = 5, AG_OPT_EWALD_OPEN = 6, AG_OPT_ADJOINT_OPEN = 7, AG_OPT_MEM_LIMIT = 8,
       AG_OPT_GROUP_SPLIT = 9, AG_OPT_GROUP_PACK = 10 };
int ag_set_option(ag_ctx *ctx, int32_t option, int64_t value);

/* Per-particle softening lengths (Sec. 3: the paper's runs soften each
 * element with its own, adaptive, length; here the lengths are given, for
 * instance by ag_neighbour_lengths from the previous tree).
 * h (n,) device FP64 in input order, copied at once (the caller may reuse
 * it after the stream passes this call).  Every pair's kernel is then the
 * mean of its two particles' M4 kernels, f = (f(r, h_i) + f(r, h_j)) / 2 and
 * likewise D, so pair forces stay equal and opposite; a tree node acts as a
 * multipole only beyond the largest length among its particles and the
 * group's targets.  Applies to trees built after the call and to
 * ag_grav_direct; the eps argument of the evaluations is then only
 * validated.  A later build or direct sum over a different number of
 * particles gives AG_ESTATE; ag_grav_backward on such a tree gives
 * AG_ESTATE.  Lengths that are not positive and finite raise the device
 * flag (AG_ENONFINITE at the next sync).  h = NULL or n = 0 returns to one
 * length per evaluation (eps). */
int ag_set_softening(ag_ctx *ctx, int64_t n, const double *h);

/* Relative opening test (Sec. 3: the paper's code opens tree nodes by the
 * geometric criterion together with the relative criterion of Springel
 * 2005).  With alpha > 0 every later forward walk (ag_grav_eval,
 * ag_grav_eval_batched) uses a node, besides the geometric test, only where
 * G M L^2 / r^4 <= alpha |a_old| (M the node's mass, L its largest box side,
 * r the distance from its centre of mass to the target) and the target lies
 * outside the cube of side 1.2 L about the centre of the node's box; a target
 * group takes its nearest point and its smallest |a_old|, so each target
 * opens at least as much as it would alone.  acc (n, 3) device FP64 in input
 * order: the accelerations of the previous evaluation; their sizes are
 * copied at once (rounded down to FP32), so the caller may overwrite acc.
 * A target with |a_old| = 0 opens every node (direct summation).  An
 * evaluation over a tree of another n gives AG_ESTATE, and so does
 * ag_grav_backward while the test is on.  Non-finite sizes raise the device
 * flag (AG_ENONFINITE at the next sync).  alpha = 0, acc = NULL or n = 0
 * turns the test off.  alpha < 0 or non-finite: AG_EINVAL. */
int ag_set_relative_opening(ag_ctx *ctx, double alpha, int64_t n, const double *acc);

/* Adaptive softening lengths from the built tree (Sec. 3: each element's
 * softening follows the local spacing; here that spacing is the distance to
 * the k-th nearest other particle).  h (n,) device FP64, written in input
 * order: h_i = sqrt(d2_k) with d2_k the k-th smallest of
 * d2_ij = (dx^2 + dy^2) + dz^2 over j != i, d = x_j - x_i, each operation
 * rounded once in FP64, so the result is exact up to that rounding.  A tree
 * built in a periodic box (ag_set_periodic before the build) takes every
 * difference at its nearest image, d - box rint(d / box), from the
 * positions as the tree holds them (wrapped into [0, box)).  The output can
 * go straight to ag_set_softening.  Each length is multiplied by scale
 * (> 0 and finite; 1 gives the distance itself).  Needs a tree from
 * ag_tree_build; a batched tree gives AG_ESTATE.  k must be in [1, 64] and
 * below n (AG_EINVAL).  Coincident particles give h = 0. */
int ag_neighbour_lengths(ag_ctx *ctx, int32_t k, double scale, double *h);

/* Fully adaptive softening with the conservative correction of Price &
 * Monaghan (2007), the form of adaptive softening the paper's runs use
 * (Sec. 3).  Kernel: the cubic spline of support h, W(r, h) = 8/(pi h^3)
 * w(r/h), w = 1 - 6u^2 + 6u^3 (u < 1/2), 2(1 - u)^3 (u < 1); psi(u)/h is
 * the potential of a unit mass spread by W (-1/r outside the support).
 * Open boundaries and an unbatched tree only (AG_ESTATE otherwise);
 * n_ngb > 32/3 and below 32 n/3 (AG_EINVAL).
 *
 * ag_pm_lengths: h_i with 1 + sum_{j != i} w(r_ij / h_i) = 3 n_ngb / 32
 * (a number density of n_ngb particles per 4/3 pi h^3) and
 * Omega_i = -(32 / (9 n_ngb)) sum_j u w'(u), u = r_ij / h_i, each h_i to a
 * relative 2e-14 or better (safeguarded Newton).  Supports holding more
 * than the 64 nearest neighbours are solved by further walks over those
 * particles alone.  h, omega (n,) device FP64, input order; synchronises
 * (AG_EHIP if a length has not settled after 256 walks).  Needs a tree from
 * ag_tree_build (any softening). */
int ag_pm_lengths(ag_ctx *ctx, double n_ngb, double *h, double *omega);

/* ag_pm_factors: Z_i = (G/2) m_i h_i / (3 n_i Omega_i) sum_{j != i} m_j
 * dphi/dh(r_ij, h_i), n_i = 3 n_ngb / (4 pi h_i^3), dphi/dh the derivative
 * of psi(r/h)/h at fixed r.  The lengths are those given to
 * ag_set_softening before the tree build (AG_ESTATE if the tree was built
 * without them); omega from ag_pm_lengths.  omega, z (n,) device FP64,
 * input order. */
int ag_pm_factors(ag_ctx *ctx, double n_ngb, double G, const double *omega, double *z);

/* ag_pm_correct: the correction's acceleration, written to acc (n, 3):
 * a_i = -(1/m_i) sum_{j != i} [Z_i W'(r, h_i) + Z_j W'(r, h_j)] d / r,
 * d = x_j - x_i, W' = dW/dr; added to the softened gravity of the same
 * lengths it gives the acceleration that conserves the energy
 * (G/2) sum_i sum_{j != i} m_i m_j psi(r_ij / h_i) / h_i.  Lengths as for
 * ag_pm_factors; z (n,) from it; coincident pairs add nothing. */
int ag_pm_correct(ag_ctx *ctx, const double *z, double *acc);

/* ag_pm_correct_add: the same correction ADDED to acc (n, 3), at the rows
 * idx[0 .. *n_idx_dev) only (idx device int32, unique; the count is read
 * on the device, as ag_adaptive_select leaves it), or at every row with
 * idx = NULL.  Only the listed rows are walked, so an adaptive step pays
 * for the rows it refreshes.  The factors z must cover every particle. */
int ag_pm_correct_add(ag_ctx *ctx, const double *z, const int32_t *idx, const int64_t *n_idx_dev,
                      double *acc);

/* Periodic boundaries (Sec. 3.4: the periodic problem's gravity uses Ewald
 * sums, its jerk only the nearest image).  box > 0 makes every later
 * ag_grav_eval, ag_grav_eval_batched and (ewald = 0 only) ag_grav_direct on
 * this context periodic in a cube of side box; positions may lie in any
 * image.  Tree builds after the call hold every position in [0, box)^3;
 * evaluating a tree built under another box gives AG_ESTATE (rebuild it).
 *   ewald = 0: every pair at its nearest image, d -> d - box * rint(d / box)
 *              per axis, for g, j and T alike.
 *              The tree opening test then also requires, per axis, all of a
 *              node's box to lie within half a box side of all of the
 *              group's box, so every particle of an accepted node shares
 *              one image.
 *   ewald = 1: g and T of all periodic images with a neutralising uniform
 *              background (Ewald's method, alpha = 2 / box), j at the
 *              nearest image.  The forward walk takes every source at its
 *              image about an origin o (the group centre rounded to a
 *              multiple of box / 2, so no node below the root straddles
 *              the planes where those images change); a second walk adds
 *              the images' correction dg = g_periodic - g_single_image (and
 *              dT) at the same images, from a table built on the device
 *              (spacing box / 64, second-order expansion about the nearest
 *              table point).  There nodes act through mass and quadrupole
 *              under an opening angle (AG_OPT_EWALD_OPEN) taken against the
 *              group's other images, and a group whose half extent is at
 *              most box / 32 sums the correction once and expands it to
 *              second order about its centre.  The sum includes each
 *              target's own images (its background tide, 4 pi G m / 3 box^3
 *              per axis).  ag_grav_direct then returns AG_ESTATE (theta = 0
 *              in ag_grav_eval is the direct sum).
 * box = 0 (with ewald = 0) restores open boundaries, the default.  While a box is set, ag_grav_backward returns
 * AG_ESTATE.  box < 0 or not finite, ewald not 0 or 1, or ewald with
 * box = 0 give AG_EINVAL. */
int ag_set_periodic(ag_ctx *ctx, double box, int32_t ewald);

/* HIP-graph capture of a call sequence on the context's stream (which must
 * not be the legacy default stream).  Between ag_graph_begin and
 * ag_graph_end, library calls are recorded, not run; device buffers they
 * need must already exist (run the same sequence once before capturing).
 * ag_graph_replay launches the recorded sequence again on the stream with
 * the same pointers (refill the input arrays in place between replays).
 * Timing must be disabled while capturing.  A call that would grow a
 * library buffer during the capture fails with AG_ESTATE; if a later call
 * outside the capture grows one (moving it), ag_graph_replay refuses with
 * AG_ESTATE until the sequence is captured again.  Calls whose count or
 * time changes from step to step take it from device memory
 * (ag_grav_eval_dev, ag_grav_timestep_dev, ag_grav_predict_age, with the
 * count from ag_adaptive_select), so one captured adaptive step can be
 * replayed for every later step. */
int ag_graph_begin(ag_ctx *ctx);
int ag_graph_end(ag_ctx *ctx);
int ag_graph_replay(ag_ctx *ctx);

/* Per-phase GPU timing.  While enabled, every library call records HIP
 * events on the context's stream around each phase it launches; the
 * accumulated milliseconds per phase (and launch counts) are returned by the
 * synchronising ag_timing_read, which also resets them when reset != 0.
 * Phases, in array order: AG_PHASE_BUILD (keys, sort, topology, moments),
 * AG_PHASE_GROUPS (active rows -> walk groups), AG_PHASE_WALK (forward
 * walk kernel only), AG_PHASE_DIRECT, AG_PHASE_STEP (timestep, select,
 * predict), AG_PHASE_ADJOINT (adjoint walk kernel only), AG_PHASE_EWALD
 * (the periodic images' correction walk), AG_PHASE_NEIGHBOUR (the
 * neighbour-length walk kernel only). */
enum { AG_PHASE_BUILD = 0, AG_PHASE_GROUPS, AG_PHASE_WALK, AG_PHASE_DIRECT, AG_PHASE_STEP,
       AG_PHASE_ADJOINT, AG_PHASE_EWALD, AG_PHASE_NEIGHBOUR, AG_NPHASE };
int ag_timing_enable(ag_ctx *ctx, int enable);
int ag_timing_read(ag_ctx *ctx, double *ms /* [AG_NPHASE] */, int64_t *launches /* [AG_NPHASE], nullable */,
                   int reset);

/* ---- oct-tree (Sec. 3: Barnes-Hut tree code) ---------------------------- */

/* Build the oct-tree over all n particles.  x, v: (n,3); m: (n,).
 * Particles are ordered along a 63-bit Morton curve (21 bits per axis) of
 * the bounding cube; a cell is split while it holds more than n_leaf
 * particles (1 <= n_leaf <= 64), down to level 21.  Each node stores FP64
 * mass, centre of mass, mean velocity, traceless quadrupole
 * Q = sum m (3 y y^T - |y|^2 I) and its rate, and its bounding box.
 * The tree, and sorted copies of x, v, m, belong to the context and stay
 * valid until the next build or refit; the caller's arrays are not kept. */
int ag_tree_build(ag_ctx *ctx, int64_t n, const double *x, const double *v, const double *m,
                  int32_t n_leaf);

/* One build over n_sys independent systems stored back to back:
 * sys_offsets is a DEVICE int64 array of n_sys + 1 non-decreasing row
 * offsets (sys_offsets[0] = 0, sys_offsets[n_sys] = n).  Systems never
 * interact.  1 <= n_sys <= 512. */
int ag_tree_build_batched(ag_ctx *ctx, int64_t n, const double *x, const double *v,
                          const double *m, int32_t n_sys, const int64_t *sys_offsets,
                          int32_t n_leaf);

/* Recompute every node's moments and bounding box from new x, v, m of the
 * same n particles, keeping the topology of the last build (the opening
 * test uses the refitted boxes, so the result stays a valid tree walk). */
int ag_tree_refit(ag_ctx *ctx, const double *x, const double *v, const double *m);

/* Synchronising query of the current tree: number of nodes and deepest level. */
int ag_tree_info(ag_ctx *ctx, int64_t *n_nodes, int32_t *max_level);

/* Copy the current tree into caller DEVICE buffers (inspection and tests).
 * Nodes are in depth-first pre-order (a node's first child is the next node).
 *   link    (n_nodes, 4) int32: skip (first node after the subtree), first
 *           sorted position, particle count, level | 0x100 for leaves
 *   moments (n_nodes, 25) double: M, centre of mass (3), mean velocity (3),
 *           Q (6), dQ/dt (6), box min (3), box max (3); tensors xx yy zz xy xz yz
 *   perm    (n,) int32: input row of each sorted position
 * Any pointer may be NULL; cap is the row capacity of link and moments
 * (AG_EINVAL if smaller than n_nodes). */
int ag_tree_export(ag_ctx *ctx, int64_t cap, int32_t *link, double *moments, int32_t *perm);

/* ---- gravity evaluation ------------------------------------------------- */

/* Tree gravity at the particles listed in active_idx (n_active entries;
 * NULL = all n particles, in which case n_active must equal n; n_active = 0
 * evaluates nothing and returns AG_OK, with active_idx NULL or not).
 * Writes rows active_idx[k] of acc (n,3), jerk (n,3), tidal (n,6); all other
 * rows are left untouched.  Any of the three outputs may be NULL to skip it.
 *
 * acc   g_i = G sum_j m_j f(r) d_ij            (d_ij = x_j - x_i)
 * jerk  j_i = dg_i/dt, the particle form of the paper's jerk integral (Eq. 5)
 * tidal T_i = grad g at x_i, whose Frobenius norm sets the tidal timestep (Eq. 7)
 *
 * Opening test (Sec. 3, geometric Barnes-Hut criterion): a node of extent L
 * (longest side of its bounding box) is used as a multipole for a group of
 * up to 64 targets only if L <= theta * r for every point of the group's
 * bounding box, r measured to the node's centre of mass, and the node's box
 * lies at least eps from the group's box.  Accepted nodes act through their
 * monopole and quadrupole (acceleration and tide) and through the mean
 * velocity plus the quadrupole rate (jerk); opened leaves act pairwise.
 * theta = 0 opens every node: direct summation.  Pair terms run in FP32 on
 * coordinates relative to the group centre, accumulated in FP64.
 * The tree must have been built (or refitted) on this context. */
int ag_grav_eval(ag_ctx *ctx, const int32_t *active_idx, int64_t n_active, double theta,
                 double eps, double G, double *acc, double *jerk, double *tidal);

/* ag_grav_eval with the number of listed rows read on the device: rows
 * active_idx[0 .. *n_active_dev), the count ag_adaptive_select writes (the
 * update set of Eq. 4 never visits the host).  active_idx and n_active_dev
 * are device memory, active_idx of capacity n (the tree's); a count outside
 * [0, n] raises the device flag (AG_EDEVICE at the next sync) and evaluates
 * nothing.  n_total (device int64, nullable) gains the count: a running
 * total of force evaluations kept on the device.  Otherwise as ag_grav_eval,
 * and free of host synchronisation, so it may be captured in a graph. */
int ag_grav_eval_dev(ag_ctx *ctx, const int32_t *active_idx, const int64_t *n_active_dev, double theta,
                     double eps, double G, double *acc, double *jerk, double *tidal, int64_t *n_total);

/* Batched variant after ag_tree_build_batched: active_idx lists global rows;
 * each target only feels its own system. */
int ag_grav_eval_batched(ag_ctx *ctx, const int32_t *active_idx, int64_t n_active,
                         double theta, double eps, double G, double *acc, double *jerk,
                         double *tidal);

/* Direct summation over all n sources (no tree needed) at the rows listed in
 * active_idx (NULL = all).  precision = AG_FP64: every operation in FP64;
 * AG_FP32_PAIRS: pair terms in FP32 on relative coordinates, FP64 sums. */
int ag_grav_direct(ag_ctx *ctx, int64_t n, const double *x, const double *v, const double *m,
                   const int32_t *active_idx, int64_t n_active, double eps, double G,
                   int precision, double *acc, double *jerk, double *tidal);

/* ag_grav_direct for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, checks and kernels, and bit-identical results, but the
 * call allocates nothing.  Its scratch (the per-split sums of a target set
 * too small to fill the device, 384 KiB) is a fixed array of the library on
 * each device, looked up when the first context on that device is created;
 * the launch shape bounds
 * the scratch for every n and n_active, so no size is refused (a larger
 * need would give AG_EINVAL).  Every call on one device shares that array:
 * calls that overlap on one device (other streams, other contexts, other
 * threads) race, so order them on one stream.  Not recorded by the phase
 * timing. */
int ag_grav_direct_noalloc(ag_ctx *ctx, int64_t n, const double *x, const double *v, const double *m,
                           const int32_t *active_idx, int64_t n_active, double eps, double G, int precision,
                           double *acc, double *jerk, double *tidal);

/* ---- timestep, bookkeeping, predictor (Sec. 2, Sec. 3) ------------------- */

/* Tidal timestep (Eq. 7) dt_grav = sqrt(eta) (|T|_F^2 / 6)^(-1/4) and its
 * power-of-two bin: the smallest k >= 0 with dt_max 2^-k <= dt_grav, clamped
 * to [0, k_max]; |T| = 0 gives dt_grav = +inf and k = 0; a non-finite T
 * gives k = k_max.  The bin is decided exactly: with
 *   n2 = (Txx^2 + Tyy^2 + Tzz^2) + 2 (Txy^2 + Txz^2 + Tyz^2),
 *   Q  = (n2 * (dt_max^2)^2) / (6 eta^2)  [each operation rounded once],
 * k is the least k with Q <= 16^k.  Rows processed: idx[0..n_idx) (device
 * int32) or, with idx = NULL and n_idx = n, all n rows; n_idx = 0 processes
 * none.  tidal (n,6) in; dt_grav (n,)
 * and bin (n,) int8 out (rows not processed are untouched). */
int ag_grav_timestep(ag_ctx *ctx, int64_t n, const int32_t *idx, int64_t n_idx,
                     const double *tidal, double eta, double dt_max, int32_t k_max,
                     double *dt_grav, int8_t *bin);

/* ag_grav_timestep over rows idx[0 .. *n_idx_dev) (idx device int32 of
 * capacity n, the count in device memory; a count outside [0, n] raises the
 * device flag and processes none). */
int ag_grav_timestep_dev(ag_ctx *ctx, int64_t n, const int32_t *idx, const int64_t *n_idx_dev,
                         const double *tidal, double eta, double dt_max, int32_t k_max, double *dt_grav,
                         int8_t *bin);

/* Force-age bookkeeping (Eq. 3, Eq. 4) for all n particles at the start of
 * a step.  Time is integer: one tick is the step of bin tick_bin, so bin k
 * spans 2^(tick_bin - min(k, tick_bin)) ticks.  For each particle:
 *   tf += step_ticks;  due iff tf >= q_f * span (Eq. 4, inclusive);
 *   a due particle gets tf = 0 (it is re-evaluated now).
 * tf_ticks (n,) int64 is updated in place; the due rows are written in
 * ascending order to active_idx (capacity n) and their number to the DEVICE
 * int64 *n_active_dev.  q_f = 0 marks every particle due.  If t0 (n,) is
 * non-NULL, the due rows also get t0 = t: the time their fresh force (and
 * jerk) will refer to in the predictor. */
int ag_adaptive_select(ag_ctx *ctx, int64_t n, int64_t *tf_ticks, const int8_t *bin,
                       int64_t step_ticks, int32_t tick_bin, double q_f,
                       int32_t *active_idx, int64_t *n_active_dev, double *t0, double t);

/* Kick-drift for a leapfrog integrator driving the scheme: for every row,
 * v += acc * dt_kick, then x += v * dt_drift.  x, v, acc: (n,3). */
int ag_kick_drift(ag_ctx *ctx, int64_t n, double *x, double *v, const double *acc,
                  double dt_kick, double dt_drift);

/* Jerk predictor (Eq. 6) in closed form: acc_out_i = acc0_i + jerk_i (t - t0_i)
 * with t - t0 and the product and sum each rounded once (no fused
 * multiply-add).  Equal to repeated application of Eq. 6 in exact arithmetic,
 * since the jerk only changes at a force update.  Rows with mask[i] == 0 are
 * left untouched (mask may be NULL = all rows).  acc_out may alias acc0.
 * jerk = NULL selects no predictor (acc_out = acc0, the ablation of Sec. 3.1;
 * t0 may then be NULL too). */
int ag_grav_predict(ag_ctx *ctx, int64_t n, const uint8_t *mask, const double *acc0,
                    const double *jerk, const double *t0, double t, double *acc_out);

/* The Eq. 6 predictor with the elapsed time taken from the force-age
 * counter of Eq. 3: acc_out_i = acc0_i + jerk_i (age_i * tick), age_ticks
 * (n,) int64 the counters as ag_adaptive_select leaves them (the ticks since
 * the row's last force update, 0 for the rows updated now) and tick the
 * length of one tick.  With integer times (t = k tick, t0 = k0 tick) this
 * equals ag_grav_predict bit for bit, and it takes no per-step argument, so
 * a captured step replays unchanged.  mask, jerk = NULL and aliasing as in
 * ag_grav_predict. */
int ag_grav_predict_age(ag_ctx *ctx, int64_t n, const uint8_t *mask, const double *acc0, const double *jerk,
                        const int64_t *age_ticks, double tick, double *acc_out);

/* Deepest force log the polynomial predictor takes. */
#define AG_PRED_MAX_DEPTH 4

/* Force log for the polynomial predictor, the alternative to Eq. 6 that
 * Sec. 2.2 names (log a few past g and extrapolate).  For each row r in
 * idx[0..n_idx) (device int32, unique; NULL with n_idx = n: all rows;
 * n_idx = 0: none): the logged forces
 * of r move one slot older (the oldest of `depth` slots is dropped), slot 0
 * takes (t, acc0[r]) and hist_n[r] grows by one up to depth.  Layout,
 * slot-major with slot 0 the newest: hist_a (depth, n, 3), hist_t (depth, n),
 * hist_n (n,) int32; all caller-owned device memory, zeroed by the caller
 * before the first log.  depth in [1, AG_PRED_MAX_DEPTH].  Rows out of
 * [0, n) are skipped and raise the device flag reported by the next
 * ag_sync (AG_EDEVICE). */
int ag_force_log(ag_ctx *ctx, int64_t n, const int32_t *idx, int64_t n_idx, int32_t depth,
                 const double *acc0, double t, double *hist_a, double *hist_t, int32_t *hist_n);

/* ag_force_log over rows idx[0 .. *n_idx_dev) (idx device int32 of
 * capacity n, the count in device memory; a count outside [0, n] raises the
 * device flag and logs none). */
int ag_force_log_dev(ag_ctx *ctx, int64_t n, const int32_t *idx, const int64_t *n_idx_dev, int32_t depth,
                     const double *acc0, double t, double *hist_a, double *hist_t, int32_t *hist_n);

/* Polynomial predictor (Sec. 2.2) from a log written by ag_force_log with
 * the same n and depth: for every row, the interpolating polynomial through
 * its newest logged forces, evaluated at t in Lagrange form,
 *   acc_out = sum_k g_k prod_{m != k} (t - t_m) / (t_k - t_m),
 * over at most order + 1 of them (order in [0, depth - 1]; 1 = the linear
 * predictor that removes the leading lag error), no more than the row has
 * logged, and stopping before the first slot that is not strictly older than
 * the one before it.  Rows with nothing logged, or with mask[i] == 0 (mask
 * NULL = all rows), are left untouched.  acc_out (n,3) must not alias the
 * log. */
int ag_grav_predict_poly(ag_ctx *ctx, int64_t n, const uint8_t *mask, int32_t depth, int32_t order,
                         const double *hist_a, const double *hist_t, const int32_t *hist_n, double t,
                         double *acc_out);

/* ---- adjoint -------------------------------------------------------------- */

/* Gradient of L = sum_k w_k . g_k over the listed rows (w is (n,3), read at
 * rows active_idx only) with respect to every particle's position and mass,
 * using the current tree (rebuild it if positions changed):
 *   dL/dx_k = G m_k sum_j J(d_kj) w_j + T_k w_k,   J = f I + D d d^T,
 *   dL/dm_k = -G sum_j f(r_kj) d_kj . w_j,         D = f'(r)/r,
 * with j running over the listed rows.  The sums are evaluated by a second
 * tree walk over the vector charges w (per node their sum W0, first moment
 * W1 = sum w y^T and second moment W2 = sum w y y^T about the node's centre
 * of mass); T_k comes from a fresh forward walk.  Both walks open nodes at
 * theta times AG_OPT_ADJOINT_OPEN / 100 (default 0.75 theta).
 * dLdx (n,3) and dLdm (n,) are overwritten for all n rows. */
int ag_grav_backward(ag_ctx *ctx, const int32_t *active_idx, int64_t n_active,
                     const double *w, double theta, double eps, double G,
                     double *dLdx, double *dLdm);

#ifdef __cplusplus
}
#endif
#endif /* ADAPTGRAV_H */
