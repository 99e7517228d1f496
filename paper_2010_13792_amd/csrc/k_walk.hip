// k_walk.hip -- Barnes-Hut tree walks: the forward walk (g, j, T at the
// active targets) and the adjoint walk (gradient of L = sum_k w_k . g_k).
//
// Work decomposition: the active targets, in key (Morton) order, are cut
// into groups of at most 64 consecutive targets of one system; one wave64
// (one workgroup) walks the tree once for its whole group.  Every lane owns
// one target; in a group of fewer than 64 targets each target is given
// several lanes, which share out the interaction list and add their parts
// at the end, so the wave stays full.  The opening test is applied to the group's bounding box
// (conservative: a node is accepted only if it would be for every point of
// the box), so the whole wave follows one traversal with no divergence in
// the interaction loops.
//
// Traversal: nodes are numbered in depth-first pre-order with a "skip" link
// past each subtree, so any range [a, b) of sibling subtrees can be walked
// by one cursor without a stack (test a; accept or leaf -> a = skip[a];
// open -> a = a + 1).  The 64 lanes hold 64 such cursors and test 64 nodes
// per step; a lane that opens a node hands the rest of its range to an LDS
// stack of ranges that idle lanes pop (load balancing).  Accepted nodes and
// the particles of opened leaves are appended (ballot prefix sums) to LDS
// lists; every 64 entries the wave stages them as FP32 data relative to the
// group centre in LDS and all lanes evaluate the tile (LDS broadcast reads),
// folding the FP32 tile sums into FP64 accumulators.
#include <float.h>

#include "ag_internal.h"
#include "pair.h"

namespace {

constexpr int kW = 64;          // lanes per wave = targets per group = tile size
constexpr int kPCap = 256;      // pending particle indices
constexpr int kNCap = 128;      // pending accepted nodes
constexpr int kSCap = 128;      // stacked cursor ranges
constexpr int kMaxSub = 32;     // most lanes given to one target of a small group
// boundary modes of a walk instance
constexpr int kOpen = 0;        // open boundaries
constexpr int kNear = 1;        // periodic, every pair at its nearest image
constexpr int kEwald = 2;       // periodic with Ewald sums: g and T at the images about the group
                                // centre (the correction walk uses the same ones), j at the nearest

// algorithmic operation count of one particle-particle interaction as written
// in ForwardPolicy::particles (outside the softening kernel; every add,
// subtract and multiply = 1, reciprocal square root = 1):
//   d and nu 6, r2 5, rsqrt 1, ri2 1, mf 2, mD 2, g 6, d.nu 5, s 1, j 12,
//   t 3, m f I 1, S 12                                                 = 57
constexpr int AG_WALK_PP_FLOPS = 57;
// algorithmic operation count of one particle-node interaction as written in
// node_interact (monopole + quadrupole g and T, mean-velocity + quadrupole-rate
// jerk; every add, subtract and multiply = 1, reciprocal square root = 1):
//   d and nu 6, r2 5, rsqrt 1, powers 4, P = Q d 15, d.P 5, h e hq 3, ca 2,
//   beta 4, g 12, e P 3, w 6, ca I 1, S diagonal 15, S off-diagonal 18,
//   V = Q nu + Qd d 33, d.nu 5, P.nu 5, d.Qd.d 6, cd 5, cp 1, j 24     = 179
constexpr int AG_PN_FLOPS = 179;

struct Tree {
    const double4* __restrict__ com;   // centre of mass, extent
    const float4* __restrict__ lo;
    const float4* __restrict__ hi;
    const int4* __restrict__ link;     // skip, start, count, level | leaf
    const float4* __restrict__ mp;     // 4 per node
    const double4* __restrict__ spos;  // sorted x, y, z, m
    const float4* __restrict__ svf;    // sorted vx, vy, vz, m
    const int32_t* __restrict__ perm;
    const int32_t* __restrict__ sys_root;
    const double4* __restrict__ ws;    // adjoint: sorted weights (w, 1 if charged)
    const float4* __restrict__ wf;     // adjoint: node charges, 4 per node
    const float* __restrict__ sh;      // sorted per-particle softening lengths, or null
};

struct Groups {
    const int32_t* __restrict__ act_pos;
    const int4* __restrict__ grp;      // start, count, system
    const int32_t* __restrict__ hdr;   // [0] = number of groups
};

struct WalkOut {
    double* acc;
    double* jerk;
    double* tidal;
    unsigned long long* stats;
    double G;
    int32_t* flags;
    int64_t iter_cap;   // > nodes + particles: every group finishes well within it
    int small_node;     // accepted nodes this small are summed pairwise
    bool mac_offset;    // opening test adds the centre-of-mass offset to the extent
    const float* rel_a; // relative opening test: |a| of the last evaluation per row (null: off)
    float rel_alpha;
    float rel_g;        // |G| of the relative test
    double box, box_inv;        // periodic cube side and inverse (periodic walks only)
    float boxf, boxf_inv, box_half;
    // Ewald correction table: (NE + 1)^3 points of spacing h over [0, NE h]^3,
    // 5 float4 each (dg 3, dT 6, H 10, pad), and the correction walk's limits
    const float4* etab;
    float etab_h, etab_hinv, etab_range;
    int etab_ne;
    float ewald_theta;  // correction walk: opening angle against the nearest image point
    float ewald_grp;    // groups of at most this half extent sum the correction once
    double* knn_out;    // neighbour lengths (input order)
    double knn_scale;   // ... each multiplied by this
    int knn_k;          // which neighbour
    int64_t knn_n;
    // Price & Monaghan terms (input order arrays)
    double pm_ngb;      // > 0: the neighbour walk solves the density condition
    double pm_G;
    double* pm_omega;
    const double* pm_h;
    double* pm_lo;      // bisection brackets of the lengths (input order)
    double* pm_hi;
    double* pm_cur;     // the length the next sum walk evaluates
    int* pm_active;     // sum walk: lengths still moving after it (list pass: lengths left to it)
    int32_t* pm_idx;    // list pass: the rows left to the sum walk
    double pm_hiscale;  // upper end of a bracket: this times the root's diagonal
    const double* pm_om;
    const double* pm_z;
    double* pm_zout;
    double* pm_acc;
    bool pm_add;        // correction: added to pm_acc (else written)
    double* dldx;       // adjoint outputs
    double* dldm;
    const double* tin;  // adjoint: tidal tensor rows of the charged targets
};

// group geometry shared by every lane (uniform values)
struct GroupBox {
    double cx, cy, cz;          // centre (FP64)
    double ox, oy, oz;          // origin of the source images (periodic walks; else the centre)
    float hx, hy, hz;           // half extents (rounded up)
    float lox, loy, loz, hix, hiy, hiz;   // absolute box, rounded outward
    float amin;                 // relative opening test: smallest |a| of the group's targets
};

__device__ __forceinline__ float f_dn(double d) {
    float f = (float)d;
    return (double)f > d ? nextafterf(f, -FLT_MAX) : f;
}
__device__ __forceinline__ float f_upr(double d) {
    float f = (float)d;
    return (double)f < d ? nextafterf(f, FLT_MAX) : f;
}

__device__ __forceinline__ GroupBox group_box(double x, double y, double z) {
    double mnx = x, mny = y, mnz = z;
    double mxx = x, mxy = y, mxz = z;
    mnx = ag_wave_min(mnx); mny = ag_wave_min(mny); mnz = ag_wave_min(mnz);
    mxx = ag_wave_max(mxx); mxy = ag_wave_max(mxy); mxz = ag_wave_max(mxz);
    GroupBox g;
    g.cx = 0.5 * (mnx + mxx); g.cy = 0.5 * (mny + mxy); g.cz = 0.5 * (mnz + mxz);
    g.ox = g.cx; g.oy = g.cy; g.oz = g.cz;
    g.hx = f_upr(0.5 * (mxx - mnx)); g.hy = f_upr(0.5 * (mxy - mny)); g.hz = f_upr(0.5 * (mxz - mnz));
    g.lox = f_dn(mnx); g.loy = f_dn(mny); g.loz = f_dn(mnz);
    g.hix = f_upr(mxx); g.hiy = f_upr(mxy); g.hiz = f_upr(mxz);
    return g;
}

// nearest periodic image of a separation: d - L rint(d / L)
__device__ __forceinline__ double near_img(double d, const WalkOut& O) { return d - O.box * rint(d * O.box_inv); }
__device__ __forceinline__ float near_imgf(float d, const WalkOut& O) {
    return __builtin_fmaf(-O.boxf, rintf(d * O.boxf_inv), d);
}

// Opening test for node data (com, extent, box) against the group box.
// Accept iff  L' <= theta * r_min  (r_min: distance from the node's centre of
// mass to the nearest point of the group box; L' the node's extent L, plus,
// with `offset` set, the distance from its centre of mass to the centre of
// its box, which opens lopsided nodes sooner)  and the node's box is at least
// eps away from the group box (so only Newtonian pairs are approximated).
// Periodic (kPer != 0): distances are taken at the nearest image of the node, and
// a node is accepted only if, along every axis, all of its box lies within
// half a box side of all of the group box -- then every particle-target pair
// of the node has that same nearest image, and the multipole stands for it.
template <int kPer>
__device__ __forceinline__ bool mac_accept(const GroupBox& g, const double4 c, const float4 lo, const float4 hi,
                                           float theta2, float eps2, bool offset, const WalkOut& O) {
    double cdx = c.x - g.cx, cdy = c.y - g.cy, cdz = c.z - g.cz;
    if (kPer) {   // the node's image about the image origin, seen from the group centre
        cdx = near_img(c.x - g.ox, O) + (g.ox - g.cx);
        cdy = near_img(c.y - g.oy, O) + (g.oy - g.cy);
        cdz = near_img(c.z - g.oz, O) + (g.oz - g.cz);
    }
    const float rx = fmaxf(fabsf((float)cdx) - g.hx, 0.f);
    const float ry = fmaxf(fabsf((float)cdy) - g.hy, 0.f);
    const float rz = fmaxf(fabsf((float)cdz) - g.hz, 0.f);
    const float r2 = rx * rx + ry * ry + rz * rz;
    float L = (float)c.w;
    if (offset) {
        const float ox = (float)c.x - 0.5f * (lo.x + hi.x);
        const float oy = (float)c.y - 0.5f * (lo.y + hi.y);
        const float oz = (float)c.z - 0.5f * (lo.z + hi.z);
        L += sqrtf(ox * ox + oy * oy + oz * oz);
    }
    float gx, gy, gz;
    float bx, by, bz;   // box centre offset from the group centre (at its nearest image)
    if (!kPer) {
        gx = fmaxf(fmaxf(lo.x - g.hix, g.lox - hi.x), 0.f);
        gy = fmaxf(fmaxf(lo.y - g.hiy, g.loy - hi.y), 0.f);
        gz = fmaxf(fmaxf(lo.z - g.hiz, g.loz - hi.z), 0.f);
    } else {
        // box centre offset at its nearest image, and the half extents
        bx = fabsf((float)(near_img(0.5 * ((double)lo.x + (double)hi.x) - g.ox, O) + (g.ox - g.cx)));
        by = fabsf((float)(near_img(0.5 * ((double)lo.y + (double)hi.y) - g.oy, O) + (g.oy - g.cy)));
        bz = fabsf((float)(near_img(0.5 * ((double)lo.z + (double)hi.z) - g.oz, O) + (g.oz - g.cz)));
        const float ex = 0.5f * (hi.x - lo.x) + g.hx;
        const float ey = 0.5f * (hi.y - lo.y) + g.hy;
        const float ez = 0.5f * (hi.z - lo.z) + g.hz;
        // nearest images only: one image for the whole node (the nearest-image
        // field jumps at half a box from each target, so a node across that
        // cut is opened); with Ewald sums the field of all images is smooth
        // there, and every source stands at its image about the image origin,
        // whose cut (half a box away, on a boundary of the root's children)
        // no node below the root crosses
        if (kPer == kNear && (bx + ex >= O.box_half || by + ey >= O.box_half || bz + ez >= O.box_half))
            return false;
        gx = fmaxf(bx - ex, 0.f);
        gy = fmaxf(by - ey, 0.f);
        gz = fmaxf(bz - ez, 0.f);
    }
    const float sep2 = gx * gx + gy * gy + gz * gz;
    if (!(r2 > 0.f && L * L <= theta2 * r2 && sep2 >= eps2)) return false;
    if (!O.rel_a) return true;
    // Relative test (Springel 2005) on top of the geometric one: a node of
    // mass M (hi.w) and extent Ln at distance r is used only if
    // G M Ln^2 / r^4 <= alpha |a_old|, the size its truncation error scales
    // with against a fraction of the target's last acceleration, and only if
    // the target lies outside the cube of side 1.2 Ln about the node's box
    // centre.  For a group, r is the distance from the centre of mass to the
    // group's box (r2 above) and |a_old| the smallest of its targets, so
    // every target passes; the cube must miss the whole group box.
    const float Ln = (float)c.w;
    if (!(O.rel_g * hi.w * Ln * Ln <= O.rel_alpha * g.amin * (r2 * r2))) return false;
    if (!kPer) {
        bx = fabsf((float)(0.5 * ((double)lo.x + (double)hi.x) - g.cx));
        by = fabsf((float)(0.5 * ((double)lo.y + (double)hi.y) - g.cy));
        bz = fabsf((float)(0.5 * ((double)lo.z + (double)hi.z) - g.cz));
    }
    const float e = 0.6f * Ln;
    return !(bx < e + g.hx && by < e + g.hy && bz < e + g.hz);
}

// particle-node interaction at quadrupole order.  d = node centre - target,
// nu = node velocity - target velocity, P = Q d, q = d.P:
//   g = ca d - ri5 P,                 ca = M ri3 + 2.5 q ri7
//   S = ca I - beta d d^T - ri5 Q + e (P d^T + d P^T),
//                                     beta = 3 M ri5 + 17.5 q ri9, e = 5 ri7
//   j = S nu - ri5 Qd d + 2.5 (d.Qd.d) ri7 d
//     = ca nu + cd d + cp P - ri5 V,  V = Q nu + Qd d,
//       cd = e P.nu - beta d.nu + 2.5 ri7 (d.Qd.d),  cp = e d.nu,
// with d.Qd.d = d.V - P.nu (Q is symmetric).  Accumulates g, j and S = -T
// (same convention as pair_interact); the ca I part of S is summed into
// `sca` and added to the diagonal once per tile.
__device__ __forceinline__ void node_interact(float dx, float dy, float dz, float nx, float ny, float nz,
                                              float M, const float* Q, const float* Qd, PairAcc<float>& A,
                                              float& sca) {
    // written as explicit multiply-add chains into the accumulators (the
    // compiler does not reassociate sums on its own)
    const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float ri2 = ri * ri;
    const float ri3 = ri * ri2;
    const float ri5 = ri3 * ri2;
    const float ri7 = ri5 * ri2;
    // Q = (xx yy zz xy xz yz)
    const float Px = __builtin_fmaf(Q[4], dz, __builtin_fmaf(Q[3], dy, Q[0] * dx));
    const float Py = __builtin_fmaf(Q[5], dz, __builtin_fmaf(Q[1], dy, Q[3] * dx));
    const float Pz = __builtin_fmaf(Q[2], dz, __builtin_fmaf(Q[5], dy, Q[4] * dx));
    const float q = __builtin_fmaf(dz, Pz, __builtin_fmaf(dy, Py, dx * Px));
    const float h = 2.5f * ri7;
    const float e = 5.f * ri7;
    const float hq = h * q;
    const float ca = __builtin_fmaf(M, ri3, hq);
    const float beta = ri2 * __builtin_fmaf(4.f, hq, 3.f * ca);
    const float nr5 = -ri5;
    A.ax = __builtin_fmaf(nr5, Px, __builtin_fmaf(ca, dx, A.ax));
    A.ay = __builtin_fmaf(nr5, Py, __builtin_fmaf(ca, dy, A.ay));
    A.az = __builtin_fmaf(nr5, Pz, __builtin_fmaf(ca, dz, A.az));
    const float ePx = e * Px, ePy = e * Py, ePz = e * Pz;
    const float wx = __builtin_fmaf(-beta, dx, ePx), wy = __builtin_fmaf(-beta, dy, ePy),
                wz = __builtin_fmaf(-beta, dz, ePz);
    sca += ca;
    A.sxx = __builtin_fmaf(nr5, Q[0], __builtin_fmaf(wx + ePx, dx, A.sxx));
    A.syy = __builtin_fmaf(nr5, Q[1], __builtin_fmaf(wy + ePy, dy, A.syy));
    A.szz = __builtin_fmaf(nr5, Q[2], __builtin_fmaf(wz + ePz, dz, A.szz));
    A.sxy = __builtin_fmaf(nr5, Q[3], __builtin_fmaf(ePy, dx, __builtin_fmaf(wx, dy, A.sxy)));
    A.sxz = __builtin_fmaf(nr5, Q[4], __builtin_fmaf(ePz, dx, __builtin_fmaf(wx, dz, A.sxz)));
    A.syz = __builtin_fmaf(nr5, Q[5], __builtin_fmaf(ePz, dy, __builtin_fmaf(wy, dz, A.syz)));
    const float Vx = __builtin_fmaf(Qd[4], dz, __builtin_fmaf(Qd[3], dy, __builtin_fmaf(Qd[0], dx,
                     __builtin_fmaf(Q[4], nz, __builtin_fmaf(Q[3], ny, Q[0] * nx)))));
    const float Vy = __builtin_fmaf(Qd[5], dz, __builtin_fmaf(Qd[1], dy, __builtin_fmaf(Qd[3], dx,
                     __builtin_fmaf(Q[5], nz, __builtin_fmaf(Q[1], ny, Q[3] * nx)))));
    const float Vz = __builtin_fmaf(Qd[2], dz, __builtin_fmaf(Qd[5], dy, __builtin_fmaf(Qd[4], dx,
                     __builtin_fmaf(Q[2], nz, __builtin_fmaf(Q[5], ny, Q[4] * nx)))));
    const float dn = __builtin_fmaf(dz, nz, __builtin_fmaf(dy, ny, dx * nx));
    const float Pn = __builtin_fmaf(Pz, nz, __builtin_fmaf(Py, ny, Px * nx));
    const float qd = __builtin_fmaf(dz, Vz, __builtin_fmaf(dy, Vy, __builtin_fmaf(dx, Vx, -Pn)));
    const float cd = __builtin_fmaf(h, qd, __builtin_fmaf(-beta, dn, e * Pn));
    const float cp = e * dn;
    A.jx = __builtin_fmaf(nr5, Vx, __builtin_fmaf(cp, Px, __builtin_fmaf(cd, dx, __builtin_fmaf(ca, nx, A.jx))));
    A.jy = __builtin_fmaf(nr5, Vy, __builtin_fmaf(cp, Py, __builtin_fmaf(cd, dy, __builtin_fmaf(ca, ny, A.jy))));
    A.jz = __builtin_fmaf(nr5, Vz, __builtin_fmaf(cp, Pz, __builtin_fmaf(cd, dz, __builtin_fmaf(ca, nz, A.jz))));
}

__device__ __forceinline__ void fold(PairAcc<double>& D, const PairAcc<float>& F) {
    D.ax += F.ax; D.ay += F.ay; D.az += F.az;
    D.jx += F.jx; D.jy += F.jy; D.jz += F.jz;
    D.sxx += F.sxx; D.syy += F.syy; D.szz += F.szz;
    D.sxy += F.sxy; D.sxz += F.sxz; D.syz += F.syz;
}

// LDS of one wave
template <int NT>
struct WalkLds {
    int plist[kPCap];
    int nlist[kNCap];
    int2 stack[kSCap];
    float4 tile[NT * kW];  // one staged tile of sources (layout set by the policy)
    int tidx[kW];          // sorted index of each staged particle (self exclusion)
};

struct Target {
    float tx, ty, tz;      // position relative to the group centre
    float vx, vy, vz;
    int p;                 // sorted position
    bool grp;              // Ewald correction summed once for the whole group
    float g0x, g0y, g0z;   // group centre relative to the image origin
    float h, hinv;         // the target's own softening length (per-particle softening)
};

// f and D of one softening length: the spline inside it, Newtonian beyond
__device__ __forceinline__ void soft_fd(float r2, float h, float hinv, float& f, float& D) {
    if (r2 >= h * h) {
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float ri2 = ri * ri;
        f = ri * ri2;
        D = -3.f * f * ri2;
    } else {
        spline_fd<float>(r2, hinv, f, D);
    }
}

// ---- forward: g, j and S = -T from particle masses and node multipoles ----
struct ForwardPolicy {
    static constexpr bool kSkipEmpty = false;
    static constexpr bool kOpenAll = false;
    static constexpr bool kImageMac = false;
    static constexpr bool kGroupSum = false;
    static constexpr int kWaves = 4;   // launch bound: waves per SIMD (128 registers)
    using Lds = WalkLds<5>;
    struct Acc {
        PairAcc<double> a;
        __device__ void zero() { a.zero(); }
        __device__ void add(const Acc& o) {
            a.ax += o.a.ax; a.ay += o.a.ay; a.az += o.a.az;
            a.jx += o.a.jx; a.jy += o.a.jy; a.jz += o.a.jz;
            a.sxx += o.a.sxx; a.syy += o.a.syy; a.szz += o.a.szz;
            a.sxy += o.a.sxy; a.sxz += o.a.sxz; a.syz += o.a.syz;
        }
    };
    template <int kPer>
    __device__ static void stage_particle(Lds& S, const Tree& T, const GroupBox& gb, int lane, int pk,
                                          const WalkOut& O) {
        const double4 q = T.spos[pk];
        const float4 u = T.svf[pk];
        double dx = q.x - gb.ox, dy = q.y - gb.oy, dz = q.z - gb.oz;
        if (kPer) {
            dx = near_img(dx, O);
            dy = near_img(dy, O);
            dz = near_img(dz, O);
        }
        S.tile[lane] = make_float4((float)dx, (float)dy, (float)dz, u.w);
        S.tile[kW + lane] = make_float4(u.x, u.y, u.z, T.sh ? T.sh[pk] : u.w);   // .w: softening length
        S.tidx[lane] = pk;
    }
    // The quantities of pair_interact, written as multiply-add chains into
    // the accumulators, with the m f I part of S summed once per tile.  The
    // self pair has d = 0 exactly (both sides round the same FP64 position),
    // so it always takes the softened branch, where it is dropped.  Periodic:
    // each pair is taken at its own nearest image.
    template <int kPer, bool kSoft>
    __device__ static void particles(const Lds& S, int cnt, const Target& t, Acc& acc, float h2, float hinv,
                                     int k0, int ks, const WalkOut& O) {
        PairAcc<float> F;
        F.zero();
        float smf = 0.f;
        for (int k = k0; k < cnt; k += ks) {
            const float4 q = S.tile[k];
            const float4 u = S.tile[kW + k];
            float dx = q.x - t.tx, dy = q.y - t.ty, dz = q.z - t.tz;
            if (kPer == kNear) {
                dx = near_imgf(dx, O);
                dy = near_imgf(dy, O);
                dz = near_imgf(dz, O);
            }
            const float nx = u.x - t.vx, ny = u.y - t.vy, nz = u.z - t.vz;
            const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
            float mf, mD;
            // per-particle softening: the pair is Newtonian beyond both lengths
            const float hh = kSoft ? fmaxf(t.h, u.w) : 0.f;
            if (r2 >= (kSoft ? hh * hh : h2)) {
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float ri2 = ri * ri;
                mf = q.w * (ri * ri2);
                mD = -3.f * mf * ri2;
            } else if (!kSoft) {
                float f, D;
                spline_fd<float>(r2, hinv, f, D);
                const float mj = (S.tidx[k] == t.p) ? 0.f : q.w;
                mf = mj * f;
                mD = mj * D;
            } else {
                // the mean of the target's and the source's kernels
                float f1, D1, f2, D2;
                soft_fd(r2, t.h, t.hinv, f1, D1);
                soft_fd(r2, u.w, 1.f / u.w, f2, D2);
                const float mj = (S.tidx[k] == t.p) ? 0.f : 0.5f * q.w;
                mf = mj * (f1 + f2);
                mD = mj * (D1 + D2);
            }
            F.ax = __builtin_fmaf(mf, dx, F.ax);
            F.ay = __builtin_fmaf(mf, dy, F.ay);
            F.az = __builtin_fmaf(mf, dz, F.az);
            float jdx = dx, jdy = dy, jdz = dz, jmf = mf, jmD = mD;
            if (kPer == kEwald) {
                // g and T take the image about the group centre (the Ewald
                // correction is summed at the same one); the jerk keeps the
                // pair's nearest image, which differs only across the cut
                const float ex = near_imgf(dx, O), ey = near_imgf(dy, O), ez = near_imgf(dz, O);
                if (ex != dx || ey != dy || ez != dz) {
                    const float r2e = __builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex));
                    const float ri = __builtin_amdgcn_rsqf(r2e);
                    jmf = q.w * (ri * ri * ri);
                    jmD = -3.f * jmf * (ri * ri);
                    jdx = ex;
                    jdy = ey;
                    jdz = ez;
                }
            }
            const float sd = jmD * __builtin_fmaf(jdz, nz, __builtin_fmaf(jdy, ny, jdx * nx));
            F.jx = __builtin_fmaf(sd, jdx, __builtin_fmaf(jmf, nx, F.jx));
            F.jy = __builtin_fmaf(sd, jdy, __builtin_fmaf(jmf, ny, F.jy));
            F.jz = __builtin_fmaf(sd, jdz, __builtin_fmaf(jmf, nz, F.jz));
            const float tx = mD * dx, ty = mD * dy, tz = mD * dz;
            smf += mf;
            F.sxx = __builtin_fmaf(tx, dx, F.sxx);
            F.syy = __builtin_fmaf(ty, dy, F.syy);
            F.szz = __builtin_fmaf(tz, dz, F.szz);
            F.sxy = __builtin_fmaf(tx, dy, F.sxy);
            F.sxz = __builtin_fmaf(tx, dz, F.sxz);
            F.syz = __builtin_fmaf(ty, dz, F.syz);
        }
        F.sxx += smf;
        F.syy += smf;
        F.szz += smf;
        fold(acc.a, F);
    }
    template <int kPer>
    __device__ static void stage_node(Lds& S, const Tree& T, const GroupBox& gb, int lane, int nk,
                                      const WalkOut& O) {
        const double4 c = T.com[nk];
        const float4 m0 = T.mp[4 * nk], m1 = T.mp[4 * nk + 1], m2 = T.mp[4 * nk + 2], m3 = T.mp[4 * nk + 3];
        float4* d = S.tile;
        double dx = c.x - gb.ox, dy = c.y - gb.oy, dz = c.z - gb.oz;
        if (kPer) {   // the opening test guarantees one image for the whole node
            dx = near_img(dx, O);
            dy = near_img(dy, O);
            dz = near_img(dz, O);
        }
        d[lane] = make_float4((float)dx, (float)dy, (float)dz, m0.x);
        d[kW + lane] = make_float4(m0.y, m0.z, m0.w, m1.x);       // u, Qxx
        d[2 * kW + lane] = make_float4(m1.y, m1.z, m1.w, m2.x);   // Qyy Qzz Qxy Qxz
        d[3 * kW + lane] = make_float4(m2.y, m2.z, m2.w, m3.x);   // Qyz, Qd xx yy zz
        d[4 * kW + lane] = make_float4(m3.y, m3.z, m3.w, 0.f);    // Qd xy xz yz
    }
    __device__ static void nodes(const Lds& S, int cnt, const Target& t, Acc& acc, int k0, int ks, const WalkOut&) {
        PairAcc<float> F;
        F.zero();
        float sca = 0.f;
        const float4* d = S.tile;
        for (int k = k0; k < cnt; k += ks) {
            const float4 a0 = d[k], a1 = d[kW + k], a2 = d[2 * kW + k], a3 = d[3 * kW + k], a4 = d[4 * kW + k];
            const float Q[6] = {a1.w, a2.x, a2.y, a2.z, a2.w, a3.x};
            const float Qd[6] = {a3.y, a3.z, a3.w, a4.x, a4.y, a4.z};
            node_interact(a0.x - t.tx, a0.y - t.ty, a0.z - t.tz, a1.x - t.vx, a1.y - t.vy, a1.z - t.vz, a0.w, Q, Qd,
                          F, sca);
        }
        F.sxx += sca;
        F.syy += sca;
        F.szz += sca;
        fold(acc.a, F);
    }
    static __device__ void wave_sum(Acc&) {}
    __device__ static void finish(const Tree& T, const WalkOut& O, const Acc& A, int p, const Target&) {
        const PairAcc<double>& acc = A.a;
        const int64_t i = T.perm[p];
        const double G = O.G;
        if (O.acc) {
            O.acc[3 * i] = G * acc.ax; O.acc[3 * i + 1] = G * acc.ay; O.acc[3 * i + 2] = G * acc.az;
        }
        if (O.jerk) {
            O.jerk[3 * i] = G * acc.jx; O.jerk[3 * i + 1] = G * acc.jy; O.jerk[3 * i + 2] = G * acc.jz;
        }
        if (O.tidal) {
            double* tt = O.tidal + 6 * i;
            tt[0] = -G * acc.sxx; tt[1] = -G * acc.syy; tt[2] = -G * acc.szz;
            tt[3] = -G * acc.sxy; tt[4] = -G * acc.sxz; tt[5] = -G * acc.syz;
        }
    }
};

// ---- adjoint: V = sum_j J(d) w_j and s = sum_j f d.w_j over vector charges ----
// For a node with charge sum W0 = sum w and first moment W1_bc = sum w_b y_c
// (y = position - node centre of mass), to first order in y:
//   V = f W0 + D (d.W0) d + D (W1 d + W1^T d + tr(W1) d) + E (d.W1.d) d
//   s = f d.W0 + f tr(W1) + D (d.W1.d)
// with f = r^-3, D = f'/r = -3 r^-5, E = D'/r = 15 r^-7 (nodes are only used
// at separations beyond the softening length).
struct AdjAccF {
    float vx, vy, vz, s;
};
struct AdjointPolicy {
    static constexpr bool kSkipEmpty = true;   // nodes without charge add nothing
    static constexpr bool kOpenAll = false;
    static constexpr bool kImageMac = false;
    static constexpr bool kGroupSum = false;
    static constexpr int kWaves = 4;   // launch bound: waves per SIMD (128 registers)
    using Lds = WalkLds<9>;
    struct Acc {
        double vx, vy, vz, s;
        __device__ void zero() { vx = vy = vz = s = 0.0; }
        __device__ void add(const Acc& o) { vx += o.vx; vy += o.vy; vz += o.vz; s += o.s; }
    };
    template <int kPer>
    __device__ static void stage_particle(Lds& S, const Tree& T, const GroupBox& gb, int lane, int pk,
                                          const WalkOut&) {
        static_assert(!kPer, "the adjoint walk has no periodic form");
        const double4 q = T.spos[pk];
        const double4 w = T.ws[pk];
        S.tile[lane] = make_float4((float)(q.x - gb.cx), (float)(q.y - gb.cy), (float)(q.z - gb.cz), 0.f);
        S.tile[kW + lane] = make_float4((float)w.x, (float)w.y, (float)w.z, 0.f);
        S.tidx[lane] = pk;
    }
    template <int kPer, bool kSoft>
    __device__ static void particles(const Lds& S, int cnt, const Target& t, Acc& acc, float h2, float hinv,
                                     int k0, int ks, const WalkOut&) {
        static_assert(!kSoft, "the adjoint walk has one softening length");
        AdjAccF F{0.f, 0.f, 0.f, 0.f};
        for (int k = k0; k < cnt; k += ks) {
            const float4 q = S.tile[k];
            const float4 w = S.tile[kW + k];
            const float dx = q.x - t.tx, dy = q.y - t.ty, dz = q.z - t.tz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            float f, D;
            if (r2 >= h2) {
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float ri2 = ri * ri;
                f = ri * ri2;
                D = -3.f * f * ri2;
            } else {
                spline_fd<float>(r2, hinv, f, D);
            }
            const float self = (S.tidx[k] == t.p) ? 0.f : 1.f;
            f *= self;
            D *= self;
            const float dw = dx * w.x + dy * w.y + dz * w.z;
            const float Ddw = D * dw;
            F.vx += f * w.x + Ddw * dx;
            F.vy += f * w.y + Ddw * dy;
            F.vz += f * w.z + Ddw * dz;
            F.s += f * dw;
        }
        acc.vx += F.vx; acc.vy += F.vy; acc.vz += F.vz; acc.s += F.s;
    }
    template <int kPer>
    __device__ static void stage_node(Lds& S, const Tree& T, const GroupBox& gb, int lane, int nk, const WalkOut&) {
        const double4 c = T.com[nk];
        float4* d = S.tile;
        d[lane] = make_float4((float)(c.x - gb.cx), (float)(c.y - gb.cy), (float)(c.z - gb.cz), 0.f);
#pragma unroll
        for (int q = 0; q < 8; ++q) d[(q + 1) * kW + lane] = T.wf[8 * nk + q];
    }
    // Second-order term with W2_bce = sum w_b y_c y_e (symmetric in c, e):
    //   V += -1/2 [105 t d/r^9 - 15 (d (d.trW + 2 d.trX) + 2 s + u)/r^7
    //              + 3 (trW + 2 trX)/r^5]
    //   s += 7.5 t/r^7 - 1.5 (d.trW + 2 d.trX)/r^5
    // u_b = W2_bce d_c d_e, s_e = W2_bce d_b d_c, t = d.u, trW_b = W2_bcc,
    // trX_c = W2_bbc.
    __device__ static void nodes(const Lds& S, int cnt, const Target& t, Acc& acc, int k0, int ks, const WalkOut&) {
        AdjAccF F{0.f, 0.f, 0.f, 0.f};
        const float4* d = S.tile;
        for (int k = k0; k < cnt; k += ks) {
            const float4 c = d[k], a0 = d[kW + k], a1 = d[2 * kW + k], a2 = d[3 * kW + k], a3 = d[4 * kW + k];
            const float4 a4 = d[5 * kW + k], a5 = d[6 * kW + k], a6 = d[7 * kW + k], a7 = d[8 * kW + k];
            // W0 = a0.xyz; W1 rows: (a1.x a1.y a1.z) (a1.w a2.x a2.y) (a2.z a2.w a3.x);
            // W2_b (xx yy zz xy xz yz): b=0 (a3.y a3.z a3.w a4.x a4.y a4.z),
            // b=1 (a4.w a5.x a5.y a5.z a5.w a6.x), b=2 (a6.y a6.z a6.w a7.x a7.y a7.z)
            const float dx = c.x - t.tx, dy = c.y - t.ty, dz = c.z - t.tz;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float ri = __builtin_amdgcn_rsqf(r2);
            const float ri2 = ri * ri;
            const float f = ri * ri2;
            const float D = -3.f * f * ri2;
            const float E = -5.f * D * ri2;
            const float W00 = a1.x, W01 = a1.y, W02 = a1.z, W10 = a1.w, W11 = a2.x, W12 = a2.y;
            const float W20 = a2.z, W21 = a2.w, W22 = a3.x;
            const float Ax = W00 * dx + W01 * dy + W02 * dz;   // W1 d
            const float Ay = W10 * dx + W11 * dy + W12 * dz;
            const float Az = W20 * dx + W21 * dy + W22 * dz;
            const float Bx = W00 * dx + W10 * dy + W20 * dz;   // W1^T d
            const float By = W01 * dx + W11 * dy + W21 * dz;
            const float Bz = W02 * dx + W12 * dy + W22 * dz;
            const float tr = W00 + W11 + W22;
            const float dWd = dx * Ax + dy * Ay + dz * Az;
            const float dW0 = dx * a0.x + dy * a0.y + dz * a0.z;
            // second moment: M_b = W2_b d (symmetric matrix times d)
            const float b0[6] = {a3.y, a3.z, a3.w, a4.x, a4.y, a4.z};
            const float b1[6] = {a4.w, a5.x, a5.y, a5.z, a5.w, a6.x};
            const float b2[6] = {a6.y, a6.z, a6.w, a7.x, a7.y, a7.z};
            const float M0x = b0[0] * dx + b0[3] * dy + b0[4] * dz, M0y = b0[3] * dx + b0[1] * dy + b0[5] * dz,
                        M0z = b0[4] * dx + b0[5] * dy + b0[2] * dz;
            const float M1x = b1[0] * dx + b1[3] * dy + b1[4] * dz, M1y = b1[3] * dx + b1[1] * dy + b1[5] * dz,
                        M1z = b1[4] * dx + b1[5] * dy + b1[2] * dz;
            const float M2x = b2[0] * dx + b2[3] * dy + b2[4] * dz, M2y = b2[3] * dx + b2[1] * dy + b2[5] * dz,
                        M2z = b2[4] * dx + b2[5] * dy + b2[2] * dz;
            const float ux = dx * M0x + dy * M0y + dz * M0z;   // u_b = d.M_b
            const float uy = dx * M1x + dy * M1y + dz * M1z;
            const float uz = dx * M2x + dy * M2y + dz * M2z;
            const float sx = dx * M0x + dy * M1x + dz * M2x;   // s = sum_b d_b M_b
            const float sy = dx * M0y + dy * M1y + dz * M2y;
            const float sz = dx * M0z + dy * M1z + dz * M2z;
            const float tt = dx * ux + dy * uy + dz * uz;
            const float tWx = b0[0] + b0[1] + b0[2], tWy = b1[0] + b1[1] + b1[2], tWz = b2[0] + b2[1] + b2[2];
            const float tXx = b0[0] + b1[3] + b2[4], tXy = b0[3] + b1[1] + b2[5], tXz = b0[4] + b1[5] + b2[2];
            const float ri5 = f * ri2, ri7 = ri5 * ri2, ri9 = ri7 * ri2;
            const float dtr = dx * (tWx + 2.f * tXx) + dy * (tWy + 2.f * tXy) + dz * (tWz + 2.f * tXz);
            const float c2 = -52.5f * tt * ri9 + 7.5f * dtr * ri7;   // coefficient of d
            const float cd = D * dW0 + D * tr + E * dWd + c2;
            F.vx += f * a0.x + cd * dx + D * (Ax + Bx) + 7.5f * ri7 * (2.f * sx + ux) - 1.5f * ri5 * (tWx + 2.f * tXx);
            F.vy += f * a0.y + cd * dy + D * (Ay + By) + 7.5f * ri7 * (2.f * sy + uy) - 1.5f * ri5 * (tWy + 2.f * tXy);
            F.vz += f * a0.z + cd * dz + D * (Az + Bz) + 7.5f * ri7 * (2.f * sz + uz) - 1.5f * ri5 * (tWz + 2.f * tXz);
            F.s += f * (dW0 + tr) + D * dWd + 7.5f * tt * ri7 - 1.5f * dtr * ri5;
        }
        acc.vx += F.vx; acc.vy += F.vy; acc.vz += F.vz; acc.s += F.s;
    }
    static __device__ void wave_sum(Acc&) {}
    __device__ static void finish(const Tree& T, const WalkOut& O, const Acc& A, int p, const Target&) {
        const int64_t i = T.perm[p];
        const double G = O.G;
        const double mi = T.spos[p].w;
        const double4 w = T.ws[p];
        double gx = G * mi * A.vx, gy = G * mi * A.vy, gz = G * mi * A.vz;
        if (w.x != 0.0 || w.y != 0.0 || w.z != 0.0) {   // target's own term T_i w_i
            const double* t = O.tin + 6 * i;
            gx += t[0] * w.x + t[3] * w.y + t[4] * w.z;
            gy += t[3] * w.x + t[1] * w.y + t[5] * w.z;
            gz += t[4] * w.x + t[5] * w.y + t[2] * w.z;
        }
        O.dldx[3 * i] = gx;
        O.dldx[3 * i + 1] = gy;
        O.dldx[3 * i + 2] = gz;
        O.dldm[i] = -G * A.s;
    }
};

// Walk the tree for one group of targets (one wave).
// ---- Ewald correction: what the periodic images add to g and T ----------
// Table lookup of the correction field of a unit mass at separation d
// (source - target): the nearest table point p of |d| (octant [0, range]^3,
// the field's symmetry supplies the signs) and its second-order expansion
//   dg(p + u) = dg - dT u - 1/2 H u u,   dT(p + u) = dT + H u,
// with H_abc = d dT_ab / d d_c (totally symmetric), tabulated exactly.
struct EwaldVal {
    float g[3];
    float t[6];    // xx yy zz xy xz yz
    float h[10];   // xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
};

template <bool kWithH>
__device__ __forceinline__ void ewald_lookup(const WalkOut& O, float dx, float dy, float dz, EwaldVal& E) {
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    if (ax > O.etab_range || ay > O.etab_range || az > O.etab_range) atomicOr(O.flags, AGF_INTERNAL);
    const int ne = O.etab_ne;
    int ix = (int)(ax * O.etab_hinv + 0.5f), iy = (int)(ay * O.etab_hinv + 0.5f), iz = (int)(az * O.etab_hinv + 0.5f);
    ix = ix < ne ? ix : ne;
    iy = iy < ne ? iy : ne;
    iz = iz < ne ? iz : ne;
    const float ux = ax - ix * O.etab_h, uy = ay - iy * O.etab_h, uz = az - iz * O.etab_h;
    const float4* q = O.etab + 5 * (((int64_t)ix * (ne + 1) + iy) * (ne + 1) + iz);
    const float4 a = q[0], b = q[1], c = q[2], d = q[3], e = q[4];
    const float Txx = a.w, Tyy = b.x, Tzz = b.y, Txy = b.z, Txz = b.w, Tyz = c.x;
    const float Hxxx = c.y, Hxxy = c.z, Hxxz = c.w, Hxyy = d.x, Hxyz = d.y, Hxzz = d.z;
    const float Hyyy = d.w, Hyyz = e.x, Hyzz = e.y, Hzzz = e.z;
    // (H u)_ab
    const float Pxx = Hxxx * ux + Hxxy * uy + Hxxz * uz;
    const float Pyy = Hxyy * ux + Hyyy * uy + Hyyz * uz;
    const float Pzz = Hxzz * ux + Hyzz * uy + Hzzz * uz;
    const float Pxy = Hxxy * ux + Hxyy * uy + Hxyz * uz;
    const float Pxz = Hxxz * ux + Hxyz * uy + Hxzz * uz;
    const float Pyz = Hxyz * ux + Hyyz * uy + Hyzz * uz;
    // dg - (dT + 1/2 H u) u
    const float gx = a.x - ((Txx + 0.5f * Pxx) * ux + (Txy + 0.5f * Pxy) * uy + (Txz + 0.5f * Pxz) * uz);
    const float gy = a.y - ((Txy + 0.5f * Pxy) * ux + (Tyy + 0.5f * Pyy) * uy + (Tyz + 0.5f * Pyz) * uz);
    const float gz = a.z - ((Txz + 0.5f * Pxz) * ux + (Tyz + 0.5f * Pyz) * uy + (Tzz + 0.5f * Pzz) * uz);
    const float sx = dx < 0.f ? -1.f : 1.f, sy = dy < 0.f ? -1.f : 1.f, sz = dz < 0.f ? -1.f : 1.f;
    E.g[0] = sx * gx;
    E.g[1] = sy * gy;
    E.g[2] = sz * gz;
    E.t[0] = Txx + Pxx;
    E.t[1] = Tyy + Pyy;
    E.t[2] = Tzz + Pzz;
    E.t[3] = sx * sy * (Txy + Pxy);
    E.t[4] = sx * sz * (Txz + Pxz);
    E.t[5] = sy * sz * (Tyz + Pyz);
    if (kWithH) {
        E.h[0] = sx * Hxxx; E.h[1] = sy * Hxxy; E.h[2] = sz * Hxxz;
        E.h[3] = sx * Hxyy; E.h[4] = sx * sy * sz * Hxyz; E.h[5] = sx * Hxzz;
        E.h[6] = sy * Hyyy; E.h[7] = sz * Hyyz; E.h[8] = sy * Hyzz; E.h[9] = sz * Hzzz;
    }
}

// The correction field dg(d) is smooth except at the lattice points n L,
// n != 0 (where the source meets another image of the target; the single
// image's own singularity at d = 0 is subtracted).  So the correction walk
// opens a node against the target group's other images: a node of extent s
// acts as a point if s <= theta_E r, r the smallest distance between the
// node's box and the group's box shifted by any n L, n != 0.  Per axis the
// gap is either the one about the group centre or, across the cut, the one
// through the neighbouring image; at least one axis takes the latter.
__device__ __forceinline__ bool ewald_accept(const GroupBox& g, const double4 c, const float4 lo, const float4 hi,
                                             const WalkOut& O) {
    float b[3], e[3];
    b[0] = fabsf((float)(near_img(0.5 * ((double)lo.x + (double)hi.x) - g.ox, O) + (g.ox - g.cx)));
    b[1] = fabsf((float)(near_img(0.5 * ((double)lo.y + (double)hi.y) - g.oy, O) + (g.oy - g.cy)));
    b[2] = fabsf((float)(near_img(0.5 * ((double)lo.z + (double)hi.z) - g.oz, O) + (g.oz - g.cz)));
    e[0] = 0.5f * (hi.x - lo.x) + g.hx;
    e[1] = 0.5f * (hi.y - lo.y) + g.hy;
    e[2] = 0.5f * (hi.z - lo.z) + g.hz;
    float s2 = 0.f, step = FLT_MAX;
    bool shifted = false;
    for (int a = 0; a < 3; ++a) {
        const float in = fmaxf(b[a] - e[a], 0.f);            // about the group centre
        const float out = fmaxf(O.boxf - b[a] - e[a], 0.f);  // through the neighbouring image
        if (out <= in) {
            s2 += out * out;
            shifted = true;
        } else {
            s2 += in * in;
            step = fminf(step, out * out - in * in);
        }
    }
    if (!shifted) s2 += step;
    return (float)c.w <= O.ewald_theta * sqrtf(s2);
}

// The correction walk: accepted nodes (and the particles of opened leaves)
// act through their mass and (on g) quadrupole at their images about the
// group centre, the
// ones the forward walk used for g and T.  A compact group (half extent at
// most ewald_grp) sums dg, dT and H over the entries once, every lane taking
// its share, and each target expands about the group centre:
//   dg(c - t) = dg(c) + dT(c) t - 1/2 H(c) t t,   dT(c - t) = dT(c) - H(c) t;
// a wider group evaluates the table at every target's own separation (the
// expansion's relative error falls as (t / |c - n L|)^3 <= (2 t / L)^3, at
// most 2.4e-4 of the correction for t <= L / 32).  The
// sum includes the target itself (dg(0) = 0; dT(0) is the tide of the
// background that neutralises its own images).
struct EwaldPolicy {
    static constexpr bool kSkipEmpty = false;
    static constexpr bool kOpenAll = false;
    static constexpr bool kImageMac = true;
    static constexpr bool kGroupSum = true;
    static constexpr int kWaves = 4;   // launch bound: waves per SIMD (128 registers)
    using Lds = WalkLds<8>;
    struct Acc {
        // g 3, T 6, (group sums only) H 10; FP32 sums of at most a few
        // thousand terms per lane: rounding ~1e-6 relative, below the table's
        float v[19];
        __device__ void zero() {
#pragma unroll
            for (int k = 0; k < 19; ++k) v[k] = 0.f;
        }
        __device__ void add(const Acc& o) {
#pragma unroll
            for (int k = 0; k < 19; ++k) v[k] += o.v[k];
        }
    };
    // entry k: tile[k] = (position about the group centre, mass), tile[kW + k]
    // and tile[2 kW + k] = traceless quadrupole xx yy zz xy | xz yz (0 for particles)
    template <int kPer>
    __device__ static void stage_particle(Lds& S, const Tree& T, const GroupBox& gb, int lane, int pk,
                                          const WalkOut& O) {
        const double4 q = T.spos[pk];
        S.tile[lane] = make_float4((float)near_img(q.x - gb.ox, O), (float)near_img(q.y - gb.oy, O),
                                   (float)near_img(q.z - gb.oz, O), (float)q.w);
        S.tile[kW + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
        S.tile[2 * kW + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    template <int kPer>
    __device__ static void stage_node(Lds& S, const Tree& T, const GroupBox& gb, int lane, int nk, const WalkOut& O) {
        const double4 c = T.com[nk];
        const float4 m0 = T.mp[4 * nk], m1 = T.mp[4 * nk + 1], m2 = T.mp[4 * nk + 2];
        S.tile[lane] = make_float4((float)near_img(c.x - gb.ox, O), (float)near_img(c.y - gb.oy, O),
                                   (float)near_img(c.z - gb.oz, O), m0.x);
        S.tile[kW + lane] = m1;
        S.tile[2 * kW + lane] = make_float4(m2.x, m2.y, 0.f, 0.f);
    }
    // Single-image Newtonian field of a mass with traceless quadrupole Q at
    // separation d (as the forward walk's node term): with P = Q d, q = d.P,
    //   g = ca d - r^-5 P,  ca = M r^-3 + 2.5 q r^-7,
    //   T = -(ca I - beta d d^T - r^-5 Q + 5 r^-7 (P d^T + d P^T)),
    //   beta = 3 M r^-5 + 17.5 q r^-9.
    __device__ static void newton_quad(float dx, float dy, float dz, float M, const float4 q0, const float4 q1,
                                       float* g, float* t) {
        const float Qxx = q0.x, Qyy = q0.y, Qzz = q0.z, Qxy = q0.w, Qxz = q1.x, Qyz = q1.y;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float ri = __builtin_amdgcn_rsqf(r2), ri2 = ri * ri;
        const float ri3 = ri * ri2, ri5 = ri3 * ri2, ri7 = ri5 * ri2, ri9 = ri7 * ri2;
        const float Px = Qxx * dx + Qxy * dy + Qxz * dz;
        const float Py = Qxy * dx + Qyy * dy + Qyz * dz;
        const float Pz = Qxz * dx + Qyz * dy + Qzz * dz;
        const float q = dx * Px + dy * Py + dz * Pz;
        const float ca = M * ri3 + 2.5f * q * ri7;
        const float beta = 3.f * M * ri5 + 17.5f * q * ri9;
        const float e = 5.f * ri7;
        g[0] = ca * dx - ri5 * Px;
        g[1] = ca * dy - ri5 * Py;
        g[2] = ca * dz - ri5 * Pz;
        t[0] = -(ca - beta * dx * dx - ri5 * Qxx + 2.f * e * Px * dx);
        t[1] = -(ca - beta * dy * dy - ri5 * Qyy + 2.f * e * Py * dy);
        t[2] = -(ca - beta * dz * dz - ri5 * Qzz + 2.f * e * Pz * dz);
        t[3] = -(-beta * dx * dy - ri5 * Qxy + e * (Px * dy + dx * Py));
        t[4] = -(-beta * dx * dz - ri5 * Qxz + e * (Px * dz + dx * Pz));
        t[5] = -(-beta * dy * dz - ri5 * Qyz + e * (Py * dz + dy * Pz));
    }
    // H_abc = dT_ab / dd_c of a point mass M at d:
    //   M (3 (d_c delta_ab + d_b delta_ac + d_a delta_bc) / r^5 - 15 d_a d_b d_c / r^7)
    __device__ static void newton_h(float dx, float dy, float dz, float M, float* h) {
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float ri = __builtin_amdgcn_rsqf(r2), ri2 = ri * ri;
        const float a = 3.f * M * ri * ri2 * ri2, b = 15.f * M * ri * ri2 * ri2 * ri2;
        const float d[3] = {dx, dy, dz};
        const int ia[10] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 2}, ib[10] = {0, 0, 0, 1, 1, 2, 1, 1, 2, 2},
                  ic[10] = {0, 1, 2, 1, 2, 2, 1, 2, 2, 2};
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            const int i = ia[q], j = ib[q], k = ic[q];
            const float del = (i == j ? d[k] : 0.f) + (i == k ? d[j] : 0.f) + (j == k ? d[i] : 0.f);
            h[q] = a * del - b * d[i] * d[j] * d[k];
        }
    }
    // A node's quadrupole adds -(1/6) Q_bc H_abc to dg (dg is harmonic away
    // from d = 0, so the trace of the second moment drops out).
    __device__ static void quad_g(const float4 q0, const float4 q1, const EwaldVal& E, float* g) {
        const float* H = E.h;   // xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
        const float Qxx = q0.x, Qyy = q0.y, Qzz = q0.z, Qxy = q0.w, Qxz = q1.x, Qyz = q1.y;
        const float c = 1.f / 6.f;
        g[0] -= c * (Qxx * H[0] + Qyy * H[3] + Qzz * H[5] + 2.f * (Qxy * H[1] + Qxz * H[2] + Qyz * H[4]));
        g[1] -= c * (Qxx * H[1] + Qyy * H[6] + Qzz * H[8] + 2.f * (Qxy * H[3] + Qxz * H[4] + Qyz * H[7]));
        g[2] -= c * (Qxx * H[2] + Qyy * H[7] + Qzz * H[9] + 2.f * (Qxy * H[4] + Qxz * H[5] + Qyz * H[8]));
    }
    __device__ static void entries(const Lds& S, int cnt, const Target& t, Acc& acc, int k0, int ks,
                                   const WalkOut& O) {
        EwaldVal E;
        if (t.grp) {
            // about the group centre: c = entry - (group centre), at its image
            // about the image origin; where that is not c's nearest image c',
            // the field continues smoothly through
            // dg(c) = dg(c') + g_single(c') - g_single(c) (likewise T and H)
            for (int k = threadIdx.x; k < cnt; k += kW) {
                const float4 e = S.tile[k];
                const float4 q0 = S.tile[kW + k], q1 = S.tile[2 * kW + k];
                const float cx = e.x - t.g0x, cy = e.y - t.g0y, cz = e.z - t.g0z;
                const float nx = near_imgf(cx, O), ny = near_imgf(cy, O), nz = near_imgf(cz, O);
                ewald_lookup<true>(O, nx, ny, nz, E);
                float gq[3] = {e.w * E.g[0], e.w * E.g[1], e.w * E.g[2]};
                float tq[6], hq[10];
#pragma unroll
                for (int c = 0; c < 6; ++c) tq[c] = e.w * E.t[c];
#pragma unroll
                for (int c = 0; c < 10; ++c) hq[c] = e.w * E.h[c];
                quad_g(q0, q1, E, gq);
                if (nx != cx || ny != cy || nz != cz) {
                    float g1[3], t1[6], g0[3], t0[6], h1[10], h0[10];
                    newton_quad(nx, ny, nz, e.w, q0, q1, g1, t1);
                    newton_quad(cx, cy, cz, e.w, q0, q1, g0, t0);
                    newton_h(nx, ny, nz, e.w, h1);
                    newton_h(cx, cy, cz, e.w, h0);
#pragma unroll
                    for (int c = 0; c < 3; ++c) gq[c] += g1[c] - g0[c];
#pragma unroll
                    for (int c = 0; c < 6; ++c) tq[c] += t1[c] - t0[c];
#pragma unroll
                    for (int c = 0; c < 10; ++c) hq[c] += h1[c] - h0[c];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) acc.v[c] += gq[c];
#pragma unroll
                for (int c = 0; c < 6; ++c) acc.v[3 + c] += tq[c];
#pragma unroll
                for (int c = 0; c < 10; ++c) acc.v[9 + c] += hq[c];
            }
        } else {
            // per target: the forward walk took g and T at d, the image about
            // the group centre; the periodic field is the same at the nearest
            // image d', where the table is accurate, so add
            // dg(d') + g_single(d') - g_single(d)  (the last two only when d' != d)
            for (int k = k0; k < cnt; k += ks) {
                const float4 e = S.tile[k];
                const float4 q0 = S.tile[kW + k], q1 = S.tile[2 * kW + k];
                const float dx = e.x - t.tx, dy = e.y - t.ty, dz = e.z - t.tz;
                const float nx = near_imgf(dx, O), ny = near_imgf(dy, O), nz = near_imgf(dz, O);
                ewald_lookup<true>(O, nx, ny, nz, E);
                float gq[3] = {e.w * E.g[0], e.w * E.g[1], e.w * E.g[2]};
                float tq[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) tq[c] = e.w * E.t[c];
                quad_g(q0, q1, E, gq);
                if (nx != dx || ny != dy || nz != dz) {
                    float g1[3], t1[6], g0[3], t0[6];
                    newton_quad(nx, ny, nz, e.w, q0, q1, g1, t1);
                    newton_quad(dx, dy, dz, e.w, q0, q1, g0, t0);
#pragma unroll
                    for (int c = 0; c < 3; ++c) gq[c] += g1[c] - g0[c];
#pragma unroll
                    for (int c = 0; c < 6; ++c) tq[c] += t1[c] - t0[c];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) acc.v[c] += gq[c];
#pragma unroll
                for (int c = 0; c < 6; ++c) acc.v[3 + c] += tq[c];
            }
        }
    }
    template <int kPer, bool kSoft>
    __device__ static void particles(const Lds& S, int cnt, const Target& t, Acc& acc, float, float, int k0,
                                     int ks, const WalkOut& O) {
        entries(S, cnt, t, acc, k0, ks, O);
    }
    __device__ static void nodes(const Lds& S, int cnt, const Target& t, Acc& acc, int k0, int ks,
                                 const WalkOut& O) {
        entries(S, cnt, t, acc, k0, ks, O);
    }
    static __device__ void wave_sum(Acc& A) {
#pragma unroll
        for (int k = 0; k < 19; ++k) {
            float v = A.v[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            A.v[k] = v;
        }
    }
    __device__ static void finish(const Tree& T, const WalkOut& O, const Acc& A, int p, const Target& t) {
        double g[3], tt[6];
        if (t.grp) {
            // the target relative to the group centre
            const double x = (double)t.tx - t.g0x, y = (double)t.ty - t.g0y, z = (double)t.tz - t.g0z;
            double H[10], Tv[6];
            for (int c = 0; c < 10; ++c) H[c] = A.v[9 + c];   // xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz
            for (int c = 0; c < 6; ++c) Tv[c] = A.v[3 + c];    // xx yy zz xy xz yz
            // (H t)_ab
            const double Pxx = H[0] * x + H[1] * y + H[2] * z, Pyy = H[3] * x + H[6] * y + H[7] * z;
            const double Pzz = H[5] * x + H[8] * y + H[9] * z, Pxy = H[1] * x + H[3] * y + H[4] * z;
            const double Pxz = H[2] * x + H[4] * y + H[5] * z, Pyz = H[4] * x + H[7] * y + H[8] * z;
            g[0] = A.v[0] + (Tv[0] - 0.5 * Pxx) * x + (Tv[3] - 0.5 * Pxy) * y + (Tv[4] - 0.5 * Pxz) * z;
            g[1] = A.v[1] + (Tv[3] - 0.5 * Pxy) * x + (Tv[1] - 0.5 * Pyy) * y + (Tv[5] - 0.5 * Pyz) * z;
            g[2] = A.v[2] + (Tv[4] - 0.5 * Pxz) * x + (Tv[5] - 0.5 * Pyz) * y + (Tv[2] - 0.5 * Pzz) * z;
            tt[0] = Tv[0] - Pxx; tt[1] = Tv[1] - Pyy; tt[2] = Tv[2] - Pzz;
            tt[3] = Tv[3] - Pxy; tt[4] = Tv[4] - Pxz; tt[5] = Tv[5] - Pyz;
        } else {
            for (int c = 0; c < 3; ++c) g[c] = A.v[c];
            for (int c = 0; c < 6; ++c) tt[c] = A.v[3 + c];
        }
        const int64_t i = T.perm[p];
        const double G = O.G;
        if (O.acc)
            for (int c = 0; c < 3; ++c) O.acc[3 * i + c] += G * g[c];
        if (O.tidal)
            for (int c = 0; c < 6; ++c) O.tidal[6 * i + c] += G * tt[c];
    }
};

// ---- the cubic spline with support 1 for the Price & Monaghan terms ----
// w(u) and w'(u) with W(r, h) = 8/(pi h^3) w(r/h); and -h^2 dphi/dh =
// psi(u) + u^2 F(u), where phi(r, h) = psi(r/h)/h is the potential of the
// spread unit mass and F = h^3 f its force kernel (the 1/u terms cancel):
//   16 u^2 - 48 u^4 + 192/5 u^5 - 14/5               (u < 1/2)
//   32 u^2 - 64 u^3 + 48 u^4 - 64/5 u^5 - 16/5        (1/2 <= u < 1), 0 beyond.
__device__ __forceinline__ double m4_w(double u) {
    return u < 0.5 ? 1.0 + u * u * (-6.0 + 6.0 * u) : (u < 1.0 ? 2.0 * (1.0 - u) * (1.0 - u) * (1.0 - u) : 0.0);
}
__device__ __forceinline__ double m4_wp(double u) {
    return u < 0.5 ? u * (-12.0 + 18.0 * u) : (u < 1.0 ? -6.0 * (1.0 - u) * (1.0 - u) : 0.0);
}
__device__ __forceinline__ double m4_dphi(double u) {
    const double u2 = u * u;
    return u < 0.5 ? u2 * (16.0 + u2 * (-48.0 + u * (192.0 / 5.0))) - 14.0 / 5.0
                   : (u < 1.0 ? u2 * (32.0 + u * (-64.0 + u * (48.0 - u * (64.0 / 5.0)))) - 16.0 / 5.0 : 0.0);
}

// One step of safeguarded Newton for S(h) = target with S increasing in h:
// s = S(h), sd = sum u w'(u) (so dS/dh = -sd / h).  The bracket [lo, hi]
// shrinks to the side of h the sign of S - target gives; the Newton point is
// taken when it falls strictly inside the bracket (growing h at most
// twofold), else twice h while h is below the root and the sum has no slope
// there, else the bracket's midpoint.
// Returns false once the length is settled, leaving hn = h: the step or the
// bracket below 2e-14 h (above the rounding noise of a sum of many terms,
// which keeps a tighter test from ever closing; Newton's last step had
// already brought h to that noise).
__device__ __forceinline__ bool pm_newton(double s, double sd, double target, double h, double& lo, double& hi,
                                          double& hn) {
    if (s < target) lo = h; else hi = h;
    hn = h;
    if (hi - lo <= 2e-14 * hi) return false;
    double t = sd < 0.0 ? h + (s - target) * h / sd : -1.0;
    // a settled Newton step is tested first: below an ulp it returns h
    // itself, which the bracket test would take for a failed step
    if (sd < 0.0 && fabs(t - h) <= 2e-14 * h) return false;
    if (s < target && t > 2.0 * h) t = 2.0 * h;
    if (!(t > lo && t < hi)) t = s < target && sd == 0.0 && 2.0 * h < hi ? 2.0 * h : 0.5 * (lo + hi);
    hn = t;
    return true;
}

// ---- k-th neighbour distance: the length fully adaptive softening follows ----
// Every node is opened; a node whose box lies farther from the group's box
// than the group's pruning radius is skipped.  Each target keeps its k
// smallest squared distances so far in registers, as an ascending list of
// kCap entries (16, 32 or 64, the smallest that holds k) whose first kCap - k
// are -inf, so the k-th sits at the fixed last place.  A candidate below it
// goes to a small buffer in LDS; when any buffer of the wave is full (and
// after every tile) the buffered values are inserted one by one with the
// branch-free network L'[i] = max(L[i-1], min(L[i], v)), whose entries are
// independent of one another (a value not below the last entry leaves the
// list as it is).  Before the walk the targets take the particles within k
// sorted positions of the group, which fills every list; the pruning radius
// is then the largest of the targets' k-th distances, and shrinks after
// every tile.  Distances are d^2 = (dx^2 + dy^2) + dz^2 with d = x_j - x_i,
// each operation rounded once.
constexpr int kKnnBuf = 8;
struct KnnLds : WalkLds<2> {
    double buf[kW * kKnnBuf];   // entry b of lane l at [b * 64 + l]
    double r2;
    int win_lo, win_hi;   // sorted positions taken before the walk
};
// kDensity: the Price & Monaghan density mode of finish (its own kernel, so
// that the plain lists keep their register budget)
template <int kCap, bool kDensity = false>
struct KnnPolicy {
    static constexpr bool kSkipEmpty = false;
    static constexpr bool kOpenAll = true;
    static constexpr bool kImageMac = false;
    static constexpr bool kGroupSum = false;
    // the list's registers: 2 kCap of them
    static constexpr int kWaves = kCap <= 16 ? 4 : (kCap <= 32 ? 3 : 1);
    using Lds = KnnLds;
    struct Acc {
        double x, y, z;   // the target
        double L[kCap];   // ascending; the last entry is the k-th so far
        int nb;           // buffered candidates
        __device__ void zero() { nb = 0; }
        __device__ void add(const Acc&) {}
    };
    // hipcc contracts a * b + c into one fma by default: not here.  In a
    // periodic tree every difference goes to its nearest image first,
    // d - L rint(d / L) (the division correctly rounded).
    template <int kPer>
    __device__ static double dist2(const double4& p, const Acc& A, const WalkOut& O) {
#pragma clang fp contract(off)
        double dx = p.x - A.x, dy = p.y - A.y, dz = p.z - A.z;
        if (kPer) {
            const double L = O.box;
            dx = dx - L * rint(dx / L);
            dy = dy - L * rint(dy / L);
            dz = dz - L * rint(dz / L);
        }
        return (dx * dx + dy * dy) + dz * dz;
    }
    __device__ static void insert(Acc& A, double v) {
#pragma unroll
        for (int i = kCap - 1; i > 0; --i) A.L[i] = fmax(A.L[i - 1], fmin(A.L[i], v));
        A.L[0] = fmin(A.L[0], v);
    }
    __device__ static void offer(Lds& S, Acc& A, double d2) {
        if (d2 < A.L[kCap - 1]) {
            S.buf[A.nb * kW + threadIdx.x] = d2;
            ++A.nb;
        }
    }
    // every lane inserts its buffered values (called by the whole wave)
    __device__ static void merge(Lds& S, Acc& A) {
        const int nbmax = ag_wave_max(A.nb);
        for (int b = 0; b < nbmax; ++b)
            insert(A, b < A.nb ? S.buf[b * kW + threadIdx.x] : __builtin_huge_val());
        A.nb = 0;
    }
    __device__ static void check_full(Lds& S, Acc& A) {
        if (__ballot(A.nb == kKnnBuf) != 0) merge(S, A);
    }
    // merge every buffer; radius^2 no target's k-th neighbour lies beyond
    __device__ static void flush(Lds& S, Acc& A, bool owner) {
        merge(S, A);
        const double r2 = ag_wave_max(owner ? A.L[kCap - 1] : 0.0);
        if (threadIdx.x == 0) S.r2 = r2;
    }
    // Both boxes are rounded outward, their gaps are exact in FP64, and the
    // relative margin covers the rounding of the squares: a skipped node
    // holds no particle at a computed d^2 <= r2.
    // Periodic: per axis the gap between two arcs of a circle of length L,
    // the centres' distance taken the short way round less both half widths
    // (every node lies inside the box, so no arc crosses the cut).
    template <int kPer>
    __device__ static double axis_gap(float lo, float hi, float glo, float ghi, const WalkOut& O) {
        if (!kPer) return fmax(fmax((double)lo - ghi, (double)glo - hi), 0.0);
        double c = fabs(0.5 * ((double)lo + hi) - 0.5 * ((double)glo + ghi));
        c = fmin(c, O.box - c);
        return fmax(c - 0.5 * (((double)hi - lo) + ((double)ghi - glo)), 0.0);
    }
    template <int kPer>
    __device__ static bool skip_node(const Lds& S, const Tree& T, const GroupBox& g, int a, const WalkOut& O) {
        const float4 lo = T.lo[a], hi = T.hi[a];
        const double gx = axis_gap<kPer>(lo.x, hi.x, g.lox, g.hix, O);
        const double gy = axis_gap<kPer>(lo.y, hi.y, g.loy, g.hiy, O);
        const double gz = axis_gap<kPer>(lo.z, hi.z, g.loz, g.hiz, O);
        return gx * gx + gy * gy + gz * gz > S.r2 * (1.0 + 1e-12);
    }
    template <int kPer>
    __device__ static void start(Lds& S, const Tree& T, const WalkOut& O, int4 gd, const Target& t, Acc& A,
                                 int part, int, int count) {
        const bool owner = part == 0;
        const double4 xi = T.spos[t.p];
        A.x = xi.x;
        A.y = xi.y;
        A.z = xi.z;
        const int k = O.knn_k;
#pragma unroll
        for (int i = 0; i < kCap; ++i) A.L[i] = i < kCap - k ? -__builtin_huge_val() : __builtin_huge_val();
        const int64_t lo = gd.x - k > 0 ? gd.x - k : 0;
        const int64_t hi = gd.x + count + k < O.knn_n ? gd.x + count + k : O.knn_n;
        if (threadIdx.x == 0) {
            S.win_lo = (int)lo;
            S.win_hi = (int)hi;
        }
        double4* P = reinterpret_cast<double4*>(S.tile);
        for (int64_t base = lo; base < hi; base += kW) {
            const int cw = hi - base < kW ? (int)(hi - base) : kW;
            __syncthreads();
            if ((int)threadIdx.x < cw) {
                P[threadIdx.x] = T.spos[base + threadIdx.x];
                S.tidx[threadIdx.x] = (int)(base + threadIdx.x);
            }
            __syncthreads();
            for (int q = 0; q < cw; ++q) {
                if (owner && S.tidx[q] != t.p) offer(S, A, dist2<kPer>(P[q], A, O));
                check_full(S, A);
            }
        }
        flush(S, A, owner);
        __syncthreads();
    }
    template <int kPer>
    __device__ static void stage_particle(Lds& S, const Tree& T, const GroupBox&, int lane, int pk, const WalkOut&) {
        reinterpret_cast<double4*>(S.tile)[lane] = T.spos[pk];
        S.tidx[lane] = pk;
    }
    template <int kPer>
    __device__ static void stage_node(Lds&, const Tree&, const GroupBox&, int, int, const WalkOut&) {}
    template <int kPer, bool kSoft>
    __device__ static void particles(Lds& S, int cnt, const Target& t, Acc& A, float, float, int k0, int,
                                     const WalkOut& O) {
        const bool owner = k0 == 0;   // the target's first lane keeps its list
        const double4* P = reinterpret_cast<const double4*>(S.tile);
        for (int q = 0; q < cnt; ++q) {
            const int pk = S.tidx[q];
            if (owner && pk != t.p && (pk < S.win_lo || pk >= S.win_hi))
                offer(S, A, dist2<kPer>(P[q], A, O));
            check_full(S, A);
        }
        flush(S, A, owner);
    }
    __device__ static void nodes(const Lds&, int, const Target&, Acc&, int, int, const WalkOut&) {}
    static __device__ void wave_sum(Acc&) {}
    // Density mode (Price & Monaghan lengths): h with S(h) = 1 + sum_i
    // w(r_i / h) = 3 N / 32 over the listed neighbours (self counted as 1),
    // by pm_newton; every particle within h is listed when the root lies
    // inside the list's last distance or the list holds all the others.
    // Also Omega = -(32 / (9 N)) sum_i u_i w'(u_i) at h.
    __device__ static void finish(const Tree& T, const WalkOut& O, const Acc& A, int p, const Target&) {
        const int64_t row = T.perm[p];
        if constexpr (!kDensity) {
            O.knn_out[row] = O.knn_scale * sqrt(A.L[kCap - 1]);
            return;
        }
        // the distances once (-1 for the leading -inf dummies)
        double r[kCap];
#pragma unroll
        for (int i = 0; i < kCap; ++i) r[i] = A.L[i] >= 0.0 ? sqrt(A.L[i]) : -1.0;
        const double target = 3.0 * O.pm_ngb / 32.0;
        auto sums = [&](double h, double& sd) {
            const double hinv = 1.0 / h;
            double sw = 1.0;
            sd = 0.0;
#pragma unroll
            for (int i = 0; i < kCap; ++i) {
                const double u = r[i] * hinv;
                if (r[i] >= 0.0 && u < 1.0) {
                    sw += m4_w(u);
                    sd += u * m4_wp(u);
                }
            }
            return sw;
        };
        const bool all = (int64_t)O.knn_k >= O.knn_n - 1;
        const double rl = r[kCap - 1];
        double hi = rl > 0.0 ? rl : 1.0, sd = 0.0;
        double shi = sums(hi, sd);
        if (all)
            for (int g = 0; g < 64 && shi < target; ++g) shi = sums(hi *= 2.0, sd);
        if (shi < target) {
            // the root lies beyond the list: the sum walk takes over from the
            // list's last distance with a bracket closed by any length at
            // which every particle counts (h = D / u*, D the root's diagonal)
            atomicOr(O.flags, AGF_PMSHORT);
            O.pm_idx[atomicAdd(O.pm_active, 1)] = (int32_t)row;
            const int root = T.sys_root[0];
            const float4 lo4 = T.lo[root], hi4 = T.hi[root];
            const double ex = (double)hi4.x - lo4.x, ey = (double)hi4.y - lo4.y, ez = (double)hi4.z - lo4.z;
            O.pm_lo[row] = hi;
            O.pm_hi[row] = O.pm_hiscale * sqrt(ex * ex + ey * ey + ez * ez);
            O.pm_cur[row] = 2.0 * hi;
            O.knn_out[row] = __builtin_nan("");
            O.pm_omega[row] = __builtin_nan("");
            return;
        }
        // start where S would meet the target if the listed neighbours filled
        // the ball of radius hi uniformly (S - 1 growing as h^3)
        double lo = 0.0, h = hi;
        if (shi > target) h = fmin(hi, hi * cbrt((target - 1.0) / (shi - 1.0)));
        for (int it = 0; it < 200; ++it) {
            const double s = sums(h, sd);
            double hn;
            if (!pm_newton(s, sd, target, h, lo, hi, hn)) break;
            h = hn;
        }
        sums(h, sd);
        O.pm_lo[row] = h;   // a closed bracket: the sum walk leaves it alone
        O.pm_hi[row] = h;
        O.knn_out[row] = h;
        O.pm_omega[row] = -(32.0 / (9.0 * O.pm_ngb)) * sd;
    }
};

// ---- Price & Monaghan sums over the pairs inside a kernel support ----
// kMode 0: Z_i = -(G m_i h_i^2 / (6 C Omega_i)) sum_{j != i, r < h_i} m_j
//          (psi + u^2 F)(r / h_i), C = 3 N / (4 pi) (number density n h^3);
// kMode 1: a_i = -(1 / m_i) sum_{j != i} [Z_i W'(r, h_i) + Z_j W'(r, h_j)] d / r
//          over r < max(h_i, h_j), W'(r, h) = 8 / (pi h^4) w'(r / h), d = x_j - x_i.
// kMode 2: one pm_newton step of a length whose support holds more
//          particles than the neighbour list: sum_j w(r / h) (self included)
//          and sum_j u w'(u) at the current h; h and Omega at h are written.
//          Targets with a closed bracket take no part; a group with none
//          left skips the whole tree.
// The lengths are the per-particle softening lengths the tree was built
// with (FP64, input order); each node's largest one (lo.w, a float) bounds
// the sources' supports in mode 1.  Coincident pairs add nothing (w'(0) = 0).
// Only the first lane of each target sums.
struct PmLds : WalkLds<2> {
    double hz[2 * kW];   // staged sources' h and Z
    double r2;           // the group's largest h^2
};
template <int kMode>
struct PmPolicy {
    static constexpr bool kSkipEmpty = false;
    static constexpr bool kOpenAll = true;
    static constexpr bool kImageMac = false;
    static constexpr bool kGroupSum = false;
    static constexpr int kWaves = 4;
    using Lds = PmLds;
    struct Acc {
        double x, y, z, m, h, zi;
        double s, ax, ay, az;
        __device__ void zero() { s = ax = ay = az = 0.0; }
        __device__ void add(const Acc&) {}
    };
    template <int kPer>
    __device__ static bool skip_node(const Lds& S, const Tree& T, const GroupBox& g, int a, const WalkOut&) {
        const float4 lo = T.lo[a], hi = T.hi[a];
        const double gx = fmax(fmax((double)lo.x - g.hix, (double)g.lox - hi.x), 0.0);
        const double gy = fmax(fmax((double)lo.y - g.hiy, (double)g.loy - hi.y), 0.0);
        const double gz = fmax(fmax((double)lo.z - g.hiz, (double)g.loz - hi.z), 0.0);
        double R2 = S.r2;
        if (kMode == 1) {
            const double hn = (double)lo.w * (1.0 + 1e-6);   // covers the float rounding of each length
            R2 = fmax(R2, hn * hn);
        }
        return gx * gx + gy * gy + gz * gz > R2 * (1.0 + 1e-12);
    }
    template <int kPer>
    __device__ static void start(Lds& S, const Tree& T, const WalkOut& O, int4, const Target& t, Acc& A, int part,
                                 int, int) {
        const double4 xi = T.spos[t.p];
        A.x = xi.x;
        A.y = xi.y;
        A.z = xi.z;
        A.m = xi.w;
        const int64_t row = T.perm[t.p];
        if (kMode == 2) {
            A.h = O.pm_lo[row] < O.pm_hi[row] ? O.pm_cur[row] : 0.0;
        } else {
            A.h = O.pm_h[row];
        }
        A.zi = kMode == 1 ? O.pm_z[row] : 0.0;
        const double r2 = ag_wave_max(part == 0 && A.h > 0.0 ? A.h * A.h : -1.0);
        if (threadIdx.x == 0) S.r2 = r2;
        __syncthreads();
    }
    template <int kPer>
    __device__ static void stage_particle(Lds& S, const Tree& T, const GroupBox&, int lane, int pk, const WalkOut& O) {
        reinterpret_cast<double4*>(S.tile)[lane] = T.spos[pk];
        S.tidx[lane] = pk;
        if (kMode == 1) {
            const int64_t row = T.perm[pk];
            S.hz[2 * lane] = O.pm_h[row];
            S.hz[2 * lane + 1] = O.pm_z[row];
        }
    }
    template <int kPer>
    __device__ static void stage_node(Lds&, const Tree&, const GroupBox&, int, int, const WalkOut&) {}
    template <int kPer, bool kSoft>
    __device__ static void particles(Lds& S, int cnt, const Target& t, Acc& A, float, float, int k0, int,
                                     const WalkOut&) {
        if (k0 != 0) return;
        const double4* P = reinterpret_cast<const double4*>(S.tile);
        constexpr double k8pi = 8.0 / 3.14159265358979323846;
        for (int q = 0; q < cnt; ++q) {
            if (kMode == 2) {   // self included: w(0) = 1
                const double4 pj = P[q];
                const double dx = pj.x - A.x, dy = pj.y - A.y, dz = pj.z - A.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < A.h * A.h) {
                    const double u = sqrt(r2) / A.h;
                    A.s += m4_w(u);
                    A.ax += u * m4_wp(u);
                }
                continue;
            }
            if (S.tidx[q] == t.p) continue;
            const double4 pj = P[q];
            const double dx = pj.x - A.x, dy = pj.y - A.y, dz = pj.z - A.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (kMode == 0) {
                if (r2 < A.h * A.h) A.s += pj.w * m4_dphi(sqrt(r2) / A.h);
            } else {
                const double hj = S.hz[2 * q], zj = S.hz[2 * q + 1];
                if (r2 > 0.0 && (r2 < A.h * A.h || r2 < hj * hj)) {
                    const double r = sqrt(r2);
                    const double hi4 = (A.h * A.h) * (A.h * A.h), hj4 = (hj * hj) * (hj * hj);
                    const double c = k8pi * (A.zi * m4_wp(r / A.h) / hi4 + zj * m4_wp(r / hj) / hj4) / r;
                    A.ax += c * dx;
                    A.ay += c * dy;
                    A.az += c * dz;
                }
            }
        }
    }
    __device__ static void nodes(const Lds&, int, const Target&, Acc&, int, int, const WalkOut&) {}
    static __device__ void wave_sum(Acc&) {}
    __device__ static void finish(const Tree& T, const WalkOut& O, const Acc& A, int p, const Target&) {
        const int64_t row = T.perm[p];
        if (kMode == 2) {
            if (!(A.h > 0.0)) return;
            double lo = O.pm_lo[row], hi = O.pm_hi[row], hn;
            if (pm_newton(A.s, A.ax, 3.0 * O.pm_ngb / 32.0, A.h, lo, hi, hn)) {
                O.pm_lo[row] = lo;
                O.pm_hi[row] = hi;
                O.pm_cur[row] = hn;
                atomicAdd(O.pm_active, 1);
            } else {
                O.pm_lo[row] = A.h;
                O.pm_hi[row] = A.h;
            }
            O.knn_out[row] = A.h;
            O.pm_omega[row] = -(32.0 / (9.0 * O.pm_ngb)) * A.ax;
        } else if (kMode == 0) {
            const double C = 3.0 * O.pm_ngb / (4.0 * 3.14159265358979323846);
            O.pm_zout[row] = -(O.pm_G * A.m * A.h * A.h / (6.0 * C * O.pm_om[row])) * A.s;
        } else if (O.pm_add) {
            O.pm_acc[3 * row] += -A.ax / A.m;
            O.pm_acc[3 * row + 1] += -A.ay / A.m;
            O.pm_acc[3 * row + 2] += -A.az / A.m;
        } else {
            O.pm_acc[3 * row] = -A.ax / A.m;
            O.pm_acc[3 * row + 1] = -A.ay / A.m;
            O.pm_acc[3 * row + 2] = -A.az / A.m;
        }
    }
};

template <class P, int kPer>
__device__ __forceinline__ bool policy_skips(const typename P::Lds& S, const Tree& T, const GroupBox& g, int a,
                                             const WalkOut& O) {
    if constexpr (P::kOpenAll) return P::template skip_node<kPer>(S, T, g, a, O);
    else if constexpr (P::kSkipEmpty) return T.wf[8 * a].w == 0.f;
    else return false;
}

template <class Pol, int kPer, bool kSoft>
__device__ __forceinline__ void walk_group(typename Pol::Lds& S, const Tree& T, const Groups& Gr, const WalkOut& O,
                                           const int4 gd, float theta2, float eps2, float h2, float hinv) {
    const int lane = threadIdx.x;
    const int count = gd.y;
    if (count <= 0) return;

    // ---- targets ----
    // A group of count < 64 targets gives each target sub = min(kMaxSub,
    // 64 / count) lanes: lane = part * count + slot, and part k of a target
    // takes every sub-th entry of each tile (lanes with part >= sub repeat
    // work that is not used).  The parts are summed at the end.
    const int sub = count * 2 > kW ? 1 : (kW / count < kMaxSub ? kW / count : kMaxSub);
    const int slot = lane % count;
    const int part = lane / count;
    // every lane holds some target of the group (no position list: all active)
    const int p_i = Gr.act_pos ? Gr.act_pos[gd.x + slot] : gd.x + slot;
    const double4 xi = T.spos[p_i];
    const float4 vi = T.svf[p_i];
    GroupBox gb = group_box(xi.x, xi.y, xi.z);
    if (kPer == kEwald) {
        // images about a multiple of half the box: its cut lies on the faces
        // of the root's children (the root of a periodic tree is the box)
        const double hb = 0.5 * O.box;
        gb.ox = hb * rint(gb.cx / hb);
        gb.oy = hb * rint(gb.cy / hb);
        gb.oz = hb * rint(gb.cz / hb);
    }
    Target tg;
    tg.tx = (float)(xi.x - gb.ox);
    tg.ty = (float)(xi.y - gb.oy);
    tg.tz = (float)(xi.z - gb.oz);
    tg.g0x = (float)(gb.cx - gb.ox);
    tg.g0y = (float)(gb.cy - gb.oy);
    tg.g0z = (float)(gb.cz - gb.oz);
    tg.h = kSoft ? T.sh[p_i] : 0.f;
    tg.hinv = kSoft ? 1.f / tg.h : 0.f;
    // multipoles only beyond every softening length of the group and the node
    const float gh2 = kSoft ? ag_wave_max(tg.h * tg.h) : eps2;
    tg.vx = vi.x;
    tg.vy = vi.y;
    tg.vz = vi.z;
    tg.p = p_i;
    tg.grp = Pol::kGroupSum && fmaxf(fmaxf(gb.hx, gb.hy), gb.hz) <= O.ewald_grp;
    gb.amin = O.rel_a ? ag_wave_min(O.rel_a[T.perm[p_i]]) : 0.f;
    typename Pol::Acc acc;
    acc.zero();
    if constexpr (Pol::kOpenAll) Pol::template start<kPer>(S, T, O, gd, tg, acc, part, slot, count);

    uint64_t n_pp = 0, n_pn = 0;

    // ---- traversal state ----
    const int root = T.sys_root[gd.z];
    int ca = 0, cb = 0;          // cursor range [ca, cb)
    int ps = 0, pc = 0;          // particles still to be listed from an opened leaf
    if (lane == 0 && root >= 0) {
        ca = root;
        cb = T.link[root].x;
    }
    int sp = 0;                  // stack depth (uniform)
    int npend = 0, ppend = 0;    // list fills (uniform)

    auto flush_particles = [&](int base, int cnt) {
        if (lane < cnt) Pol::template stage_particle<kPer>(S, T, gb, lane, S.plist[base + lane], O);
        __syncthreads();
        Pol::template particles<kPer, kSoft>(S, cnt, tg, acc, h2, hinv, part, sub, O);
        n_pp += (uint64_t)cnt;
        __syncthreads();
    };
    auto flush_nodes = [&](int base, int cnt) {
        if (lane < cnt) Pol::template stage_node<kPer>(S, T, gb, lane, S.nlist[base + lane], O);
        __syncthreads();
        Pol::nodes(S, cnt, tg, acc, part, sub, O);
        n_pn += (uint64_t)cnt;
        __syncthreads();
    };

    int64_t iters = 0;
    for (;;) {
        // every step tests a node or lists particles, so the loop ends within
        // (nodes + particles) steps; the cap only guards against a corrupt tree
        if (++iters > O.iter_cap) {
            if (lane == 0) atomicOr(O.flags, AGF_INTERNAL);
            break;
        }
        // 1. idle lanes take ranges from the stack
        {
            const bool idle = (ca >= cb) && pc == 0;
            const uint64_t im = __ballot(idle);
            const int nidle = __popcll(im);
            const int take = nidle < sp ? nidle : sp;
            if (take > 0) {
                const int r = ag_prefix_count(im);
                if (idle && r < take) {
                    const int2 e = S.stack[sp - 1 - r];
                    ca = e.x;
                    cb = e.y;
                }
                sp -= take;
            }
            __syncthreads();
        }
        const bool walking = (ca < cb) && pc == 0;
        if (__ballot(walking || pc > 0) == 0) break;

        // 2. test one node per walking lane
        int push_node = -1;
        int push_range_a = 0, push_range_b = 0;
        bool want_push = false;
        if (walking) {
            const int a = ca;
            const int4 L = T.link[a];
            const bool leaf = (L.w & 0x100) != 0;
            if (policy_skips<Pol, kPer>(S, T, gb, a, O)) {
                ca = L.x;                  // nothing below this node matters
            } else {
                const bool acc_ok =
                    Pol::kOpenAll ? false
                    : Pol::kImageMac ? ewald_accept(gb, T.com[a], T.lo[a], T.hi[a], O)
                                   : mac_accept<kPer>(gb, T.com[a], T.lo[a], T.hi[a], theta2,
                                                      kSoft ? fmaxf(gh2, T.lo[a].w * T.lo[a].w) : eps2,
                                                      O.mac_offset, O);
                if (acc_ok && L.z > O.small_node) {
                    push_node = a;
                    ca = L.x;
                } else if (acc_ok || leaf) {
                    ps = L.y;
                    pc = L.z;
                    ca = L.x;
                } else {                   // open an inner node
                    if (L.x < cb) {        // siblings remain: offer them to the stack
                        want_push = true;
                        push_range_a = L.x;
                        push_range_b = cb;
                    }
                    ca = a + 1;
                }
            }
        }
        // 3a. accepted nodes -> node list (always fits: npend < 64 here)
        {
            const uint64_t m = __ballot(push_node >= 0);
            if (m) {
                const int r = ag_prefix_count(m);
                if (push_node >= 0) S.nlist[npend + r] = push_node;
                npend += __popcll(m);
            }
        }
        // 3b. split ranges -> stack (lanes beyond capacity keep their range)
        {
            const uint64_t m = __ballot(want_push);
            if (m) {
                const int r = ag_prefix_count(m);
                const int room = kSCap - sp;
                if (want_push && r < room) {
                    S.stack[sp + r] = make_int2(push_range_a, push_range_b);
                    cb = push_range_a;
                }
                const int pushed = __popcll(m);
                sp += pushed < room ? pushed : room;
            }
        }
        // 3c. particles of opened leaves -> particle list, as room allows
        {
            const int want = pc;
            const int incl = ag_wave_incl_scan(want);
            const int excl = incl - want;
            const int total = __shfl(incl, 63, 64);
            if (total > 0) {
                const int room = kPCap - ppend;
                int give = room - excl;
                give = give < 0 ? 0 : (give > want ? want : give);
                for (int k = 0; k < give; ++k) S.plist[ppend + excl + k] = ps + k;
                ps += give;
                pc -= give;
                ppend += total < room ? total : room;
            }
        }
        __syncthreads();
        // 4. evaluate full tiles
        while (npend >= kW) {
            npend -= kW;
            flush_nodes(npend, kW);
        }
        while (ppend >= kW) {
            ppend -= kW;
            flush_particles(ppend, kW);
        }
    }
    if (npend > 0) flush_nodes(0, npend);
    if (ppend > 0) flush_particles(0, ppend);

    if (Pol::kGroupSum && tg.grp) {
        // every lane summed its own share of the entries: add all 64
        Pol::wave_sum(acc);
    } else if constexpr (Pol::kOpenAll) {
        // (the neighbour walk's parts other than the first keep nothing)
    } else if (sub > 1) {
        // sum the parts of every target in LDS (the walk lists are free now)
        static_assert(sizeof(typename Pol::Lds) >= sizeof(typename Pol::Acc) * kW, "LDS too small");
        typename Pol::Acc* red = reinterpret_cast<typename Pol::Acc*>(&S);
        __syncthreads();
        red[lane] = acc;
        __syncthreads();
        if (part == 0)
            for (int j = 1; j < sub; ++j) acc.add(red[slot + j * count]);
        __syncthreads();
    }
    if (part == 0) Pol::finish(T, O, acc, p_i, tg);
    if (lane == 0 && O.stats) {
        atomicAdd(&O.stats[0], (unsigned long long)(n_pp * (uint64_t)count));
        atomicAdd(&O.stats[1], (unsigned long long)(n_pn * (uint64_t)count));
        atomicAdd(&O.stats[2], (unsigned long long)count);
        atomicAdd(&O.stats[3], 1ull);
    }
}

// Persistent walk: each workgroup (one wave) pops groups from eight work
// queues, one per contiguous eighth of the (Morton-ordered) group list.  A
// workgroup starts on queue blockIdx % 8 -- the XCD the hardware dispatches
// it to, so spatially neighbouring groups share that XCD's L2 -- and steals
// from the other queues when its own runs dry.  The register budget is held
// to 128 VGPRs (four waves per SIMD); the few values this spills live
// outside the interaction loops.
template <class Pol, int kPer, bool kSoft = false>
__global__ void __launch_bounds__(kW, Pol::kWaves) k_walk(Tree T, Groups Gr, WalkOut O, int* __restrict__ qctr,
                                             float theta2, float eps2, float h2, float hinv) {
    __shared__ typename Pol::Lds S;
    __shared__ int s_g;
    const int n_groups = Gr.hdr[0];
    const int home = blockIdx.x & 7;
    int q = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            int g = -1;
            while (q < 8) {
                const int qq = (home + q) & 7;
                const int lo = (int)((int64_t)n_groups * qq / 8);
                const int hi = (int)((int64_t)n_groups * (qq + 1) / 8);
                const int k = atomicAdd(&qctr[qq], 1);
                if (lo + k < hi) {
                    g = lo + k;
                    break;
                }
                ++q;
            }
            s_g = g;
        }
        __syncthreads();
        const int g = s_g;
        __syncthreads();
        if (g < 0) break;
        walk_group<Pol, kPer, kSoft>(S, T, Gr, O, Gr.grp[g], theta2, eps2, h2, hinv);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Ewald correction table
// ---------------------------------------------------------------------------
// The periodic field of a unit mass (G = 1) and its images with a uniform
// neutralising background, split with alpha = 2 / L:
//   g = sum_n B(r_n) y_n + (4 pi / L^3) sum_k k / k^2 exp(-k^2 / 4 alpha^2) sin(k.d),
//   B(r) = erfc(alpha r) / r^3 + (2 alpha / sqrt(pi)) exp(-alpha^2 r^2) / r^2,
// y_n = d + n L; with C = B'/r and D = C'/r per image,
//   T_ab = -(B delta_ab + C y_a y_b),
//   H_abc = dT_ab / dd_c = -(C (y_c delta_ab + y_b delta_ac + y_a delta_bc) + D y_a y_b y_c),
// and the reciprocal terms -w k_a k_b cos(k.d), +w k_a k_b k_c sin(k.d).  The
// n = 0 image enters without its Newtonian part (B -> B - 1/r^3), by the
// series of that difference where alpha r < 1/2, so the table holds the
// correction dg = g - d / |d|^3 (and its derivatives), smooth up to d = 0.
// Images |n_a| <= 3, wave vectors |h_a| <= 4 (dropped terms below 1e-19).
__device__ void ewald_radial(double r, double alpha, bool newton_removed, double& B, double& C, double& D) {
    const double sp = 1.1283791670955126;   // 2 / sqrt(pi)
    const double z = alpha * r;
    if (newton_removed && z < 0.5) {
        // c_k = (-1)^k 2k / ((2k + 1) k!) alpha^(2k+1):  B = sp sum_{k>=1} c_k r^(2k-2),
        // C = sp sum_{k>=2} c_k (2k-2) r^(2k-4),  D = sp sum_{k>=3} c_k (2k-2)(2k-4) r^(2k-6)
        double sb = 0.0, sc = 0.0, sd = 0.0;
        double ak = alpha * alpha * alpha, fact = 1.0;
        double r2 = r * r, pb = 1.0, pc = 1.0, pd = 1.0;
        for (int k = 1; k <= 24; ++k) {
            if (k > 1) {
                ak *= alpha * alpha;
                fact *= k;
                pb *= r2;
            }
            if (k > 2) pc *= r2;
            if (k > 3) pd *= r2;
            const double c = ((k & 1) ? -1.0 : 1.0) * (2.0 * k) / ((2.0 * k + 1.0) * fact) * ak;
            sb += c * pb;
            if (k >= 2) sc += c * (2.0 * k - 2.0) * pc;
            if (k >= 3) sd += c * (2.0 * k - 2.0) * (2.0 * k - 4.0) * pd;
        }
        B = sp * sb;
        C = sp * sc;
        D = sp * sd;
        return;
    }
    const double e = exp(-z * z), ec = erfc(z);
    const double r2 = r * r, r3 = r2 * r, r4 = r2 * r2, r5 = r4 * r;
    double b = ec / r3 + sp * alpha * e / r2;
    double b1 = -3.0 * ec / r4 - sp * alpha * e * (3.0 / r3 + 2.0 * alpha * alpha / r);
    double b2 = 12.0 * ec / r5 + sp * alpha * e * (12.0 / r4 + 8.0 * alpha * alpha / r2 + 4.0 * alpha * alpha * alpha * alpha);
    if (newton_removed) {
        b -= 1.0 / r3;
        b1 += 3.0 / r4;
        b2 -= 12.0 / r5;
    }
    B = b;
    C = b1 / r;
    D = b2 / r2 - b1 / r3;
}

__global__ void k_ewald_table(double L, int ne, double h, float4* __restrict__ tab) {
    const int np = (ne + 1) * (ne + 1) * (ne + 1);
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= np) return;
    const int iz = id % (ne + 1), iy = (id / (ne + 1)) % (ne + 1), ix = id / ((ne + 1) * (ne + 1));
    const double d[3] = {ix * h, iy * h, iz * h};
    const double alpha = 2.0 / L;
    double g[3] = {0, 0, 0}, T[6] = {0, 0, 0, 0, 0, 0}, H[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    // index pairs of T and triples of H
    const int ta[6] = {0, 1, 2, 0, 0, 1}, tb[6] = {0, 1, 2, 1, 2, 2};
    const int ha[10] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 2}, hb[10] = {0, 0, 0, 1, 1, 2, 1, 1, 2, 2},
              hc[10] = {0, 1, 2, 1, 2, 2, 1, 2, 2, 2};
    for (int a = -3; a <= 3; ++a)
        for (int b = -3; b <= 3; ++b)
            for (int c = -3; c <= 3; ++c) {
                const double y[3] = {d[0] + a * L, d[1] + b * L, d[2] + c * L};
                const double r = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
                double B, C, D;
                ewald_radial(r, alpha, a == 0 && b == 0 && c == 0, B, C, D);
                for (int q = 0; q < 3; ++q) g[q] += B * y[q];
                for (int q = 0; q < 6; ++q) T[q] -= (ta[q] == tb[q] ? B : 0.0) + C * y[ta[q]] * y[tb[q]];
                for (int q = 0; q < 10; ++q) {
                    const int i = ha[q], j = hb[q], k = hc[q];
                    const double del = (i == j ? y[k] : 0.0) + (i == k ? y[j] : 0.0) + (j == k ? y[i] : 0.0);
                    H[q] -= C * del + D * y[i] * y[j] * y[k];
                }
            }
    const double pre = 4.0 * 3.14159265358979323846 / (L * L * L);
    const double kf = 2.0 * 3.14159265358979323846 / L;
    for (int a = -4; a <= 4; ++a)
        for (int b = -4; b <= 4; ++b)
            for (int c = -4; c <= 4; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                const double k[3] = {kf * a, kf * b, kf * c};
                const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                const double w = pre * exp(-k2 / (4.0 * alpha * alpha)) / k2;
                double sn, cs;
                sincos(k[0] * d[0] + k[1] * d[1] + k[2] * d[2], &sn, &cs);
                for (int q = 0; q < 3; ++q) g[q] += w * k[q] * sn;
                for (int q = 0; q < 6; ++q) T[q] -= w * k[ta[q]] * k[tb[q]] * cs;
                for (int q = 0; q < 10; ++q) H[q] += w * k[ha[q]] * k[hb[q]] * k[hc[q]] * sn;
            }
    float4* o = tab + 5 * (int64_t)id;
    o[0] = make_float4((float)g[0], (float)g[1], (float)g[2], (float)T[0]);
    o[1] = make_float4((float)T[1], (float)T[2], (float)T[3], (float)T[4]);
    o[2] = make_float4((float)T[5], (float)H[0], (float)H[1], (float)H[2]);
    o[3] = make_float4((float)H[3], (float)H[4], (float)H[5], (float)H[6]);
    o[4] = make_float4((float)H[7], (float)H[8], (float)H[9], 0.f);
}

// ---------------------------------------------------------------------------
// active rows -> groups
// ---------------------------------------------------------------------------
// A group is a run of consecutive sibling cells, each with at most 64 active
// targets, whose parent holds more than 64 (so a group never reaches beyond
// its parent cell), packed up to 64 targets; a leaf holding more than 64
// active targets (coincident points at the deepest level) is cut in chunks
// of 64.  Cells of the system-prefix levels are never packed together, so a
// group never mixes systems.
__global__ void k_fill0(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Active rows -> flags over sorted positions, without atomics: every listed
// entry k stamps k + 1 at its position, then each entry checks that its own
// stamp survived (a repeated row loses to one of its copies) and sets the flag.
// The list's length is n_act, or, with n_dev set, the count stored at *n_dev
// (at most n_act = n; a count outside [0, n] raises the flag and lists none).
__device__ __forceinline__ int64_t list_len(int64_t n_act, const int64_t* __restrict__ n_dev) {
    if (!n_dev) return n_act;
    const int64_t v = *n_dev;
    return (v < 0 || v > n_act) ? 0 : v;
}

__global__ void k_mark_stamp(int64_t n_act, const int64_t* __restrict__ n_dev, const int32_t* __restrict__ idx,
                             int64_t n, const int32_t* __restrict__ rank, int32_t* __restrict__ stamp,
                             int32_t* __restrict__ flags, int64_t* __restrict__ n_total) {
    if (n_dev && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t v = *n_dev;
        if (v < 0 || v > n_act) atomicOr(flags, AGF_BADINDEX);
        else if (n_total) *n_total += v;   // running total of evaluations
    }
    n_act = list_len(n_act, n_dev);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_act;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[k];
        if (i < 0 || i >= n) {
            atomicOr(flags, AGF_BADINDEX);
            continue;
        }
        stamp[rank[i]] = (int32_t)(k + 1);
    }
}

__global__ void k_mark_check(int64_t n_act, const int64_t* __restrict__ n_dev, const int32_t* __restrict__ idx,
                             int64_t n, const int32_t* __restrict__ rank, const int32_t* __restrict__ stamp,
                             int32_t* __restrict__ flag, int32_t* __restrict__ flags) {
    n_act = list_len(n_act, n_dev);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_act;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx[k];
        if (i < 0 || i >= n) continue;
        const int p = rank[i];
        if (stamp[p] == (int32_t)(k + 1)) flag[p] = 1;
        else atomicOr(flags, AGF_BADINDEX);
    }
}


__global__ void k_compact_pos(int64_t n, const int32_t* __restrict__ flag, const int32_t* __restrict__ off,
                              int32_t* __restrict__ out) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x)
        if (flag[p]) out[off[p]] = (int32_t)p;
}

struct GroupCtx {
    const int4* __restrict__ link;
    const int32_t* __restrict__ aoff;   // exclusive scan of the active flags over sorted positions (null: all)
    const int64_t* __restrict__ sys_off;
    int n_sys;
    int sys_levels;
    int span;   // cap on the particles of a group's cells (0 = none)
    int cap;    // targets per group (at most one wave)
    int split;  // groups of 33 .. split targets are emitted as two halves (0 = none)
    int pack;   // 1: runs of small children are cut every `cap` targets, not at child boundaries
};

__device__ __forceinline__ int sys_of_pos(const GroupCtx& C, int64_t p) {
    int lo = 0, hi = C.n_sys;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (C.sys_off[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

// Count (out == nullptr) or write the groups node `id` is responsible for.
__device__ int node_groups(const GroupCtx& C, int id, int4* __restrict__ out) {
    const int4 L = C.link[id];
    const int lvl = L.w & 0xff;
    const bool leaf = (L.w & 0x100) != 0;
    const int a0 = C.aoff ? C.aoff[L.y] : L.y;
    const int a = (C.aoff ? C.aoff[L.y + L.z] : L.y + L.z) - a0;
    const bool forced = lvl < C.sys_levels;
    // too many targets for one wave, or (span) a cell too large to be one
    // compact group even if few of its particles are active
    const bool big = forced || a > C.cap || (C.span > 0 && !leaf && L.z > C.span);
    int ng = 0;
    auto emit1 = [&](int start, int cnt, int64_t pos) {
        if (out) out[ng] = make_int4(start, cnt, C.n_sys > 1 ? sys_of_pos(C, pos) : 0, 0);
        ++ng;
    };
    // a wave gives each of k targets 64 / k lanes (whole lanes): 33 .. 42
    // targets leave a third or more of the lanes idle, two halves of 17 .. 21
    // use three lanes each
    auto emit = [&](int start, int cnt, int64_t pos) {
        if (C.split > 0 && cnt > 32 && cnt <= C.split) {
            emit1(start, cnt / 2, pos);
            emit1(start + cnt / 2, cnt - cnt / 2, pos);
        } else {
            emit1(start, cnt, pos);
        }
    };
    if (!big) {
        if (id == 0 && a > 0) emit(a0, a, L.y);   // a small whole tree is one group
        return ng;
    }
    if (leaf) {
        for (int k = 0; k < a; k += C.cap) emit(a0 + k, a - k < C.cap ? a - k : C.cap, L.y);
        return ng;
    }
    int run_start = 0, run_cnt = 0, run_span = 0;
    int64_t run_pos = 0;
    // (pack: a run, contiguous in the target order, is cut into groups of
    // `cap` targets and a remainder, which may split a child between two
    // groups; the groups stay inside this node's cell)
    auto emit_run = [&](int start, int cnt, int64_t pos) {
        if (!C.pack) {
            emit(start, cnt, pos);
            return;
        }
        for (int k = 0; k < cnt; k += C.cap) emit(start + k, cnt - k < C.cap ? cnt - k : C.cap, pos);
    };
    for (int ch = id + 1, k8 = 0; ch < L.x && k8 < 8; ch = C.link[ch].x, ++k8) {
        const int4 Lc = C.link[ch];
        const int c0 = C.aoff ? C.aoff[Lc.y] : Lc.y;
        const int ac = (C.aoff ? C.aoff[Lc.y + Lc.z] : Lc.y + Lc.z) - c0;
        const bool leafc = (Lc.w & 0x100) != 0;
        const bool bigc = (Lc.w & 0xff) < C.sys_levels || ac > C.cap || (C.span > 0 && !leafc && Lc.z > C.span);
        if (bigc || ac == 0 || forced) {
            if (run_cnt > 0) emit_run(run_start, run_cnt, run_pos);
            run_cnt = 0;
            run_span = 0;
            if (forced && !bigc && ac > 0) emit(c0, ac, Lc.y);
            continue;
        }
        if ((!C.pack && run_cnt + ac > C.cap) || (C.span > 0 && run_span + Lc.z > C.span)) {
            if (run_cnt > 0) emit_run(run_start, run_cnt, run_pos);
            run_cnt = 0;
            run_span = 0;
        }
        if (run_cnt == 0) {
            run_start = c0;
            run_pos = Lc.y;
        }
        run_cnt += ac;
        run_span += Lc.z;
    }
    if (run_cnt > 0) emit_run(run_start, run_cnt, run_pos);
    return ng;
}

// counts for every slot up to the node bound (zero past the last node)
__global__ void k_group_count(GroupCtx C, const int64_t* __restrict__ hdr, int64_t max_nodes,
                              int32_t* __restrict__ gcnt) {
    const int64_t nn = hdr[0];
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < max_nodes;
         id += (int64_t)gridDim.x * blockDim.x)
        gcnt[id] = id < nn ? node_groups(C, (int)id, nullptr) : 0;
}

__global__ void k_group_emit(GroupCtx C, const int64_t* __restrict__ hdr, const int32_t* __restrict__ goff,
                             int4* __restrict__ grp, int32_t* __restrict__ ghdr, int* __restrict__ qctr) {
    const int64_t nn = hdr[0];
    for (int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; id < nn;
         id += (int64_t)gridDim.x * blockDim.x) {
        if (goff[id + 1] > goff[id]) node_groups(C, (int)id, grp + goff[id]);
    }
    if (blockIdx.x == 0 && threadIdx.x < 8) qctr[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) ghdr[0] = goff[nn];
}

int grid_for(int64_t n, int threads = 256) {
    int64_t b = (n + threads - 1) / threads;
    if (b > 8192) b = 8192;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

int ag_prepare_groups(ag_ctx* c, const int32_t* idx, int64_t n_act, int64_t* max_groups, const int64_t* n_dev,
                      int64_t* n_total) {
    const int64_t n = c->n;
    const int64_t mg = n_act + c->n_sys + 1;   // every group holds at least one target
    AG_TRY(ag_ensure(c, c->act_flag, n * 4));
    AG_TRY(ag_ensure(c, c->act_off, (n + 1) * 4));
    AG_TRY(ag_ensure(c, c->act_pos, n * 4));
    AG_TRY(ag_ensure(c, c->grp, mg * 16));
    AG_TRY(ag_ensure(c, c->grp_hdr, (16 + AG_MAX_SYS + 1) * 4));
    AG_TRY(ag_ensure(c, c->grp_cnt, (c->max_nodes + 1) * 4));
    AG_TRY(ag_ensure(c, c->grp_off, (c->max_nodes + 1) * 4));
    PhaseScope phase(c, AG_PHASE_GROUPS);
    hipStream_t st = c->stream;
    int32_t* flag = c->act_flag.as<int32_t>();
    int32_t* off = c->act_off.as<int32_t>();
    c->all_active = idx == nullptr;
    if (idx) {
        hipLaunchKernelGGL(k_fill0, dim3(grid_for(n)), dim3(256), 0, st, flag, n);
        // the scan output doubles as the stamp array until the scan runs
        hipLaunchKernelGGL(k_mark_stamp, dim3(grid_for(n_act)), dim3(256), 0, st, n_act, n_dev, idx, n,
                           c->rank.as<int32_t>(), off, c->dflags.as<int32_t>(), n_total);
        hipLaunchKernelGGL(k_mark_check, dim3(grid_for(n_act)), dim3(256), 0, st, n_act, n_dev, idx, n,
                           c->rank.as<int32_t>(), off, flag, c->dflags.as<int32_t>());
        AG_TRY(ag_scan_i32(c, flag, off, n));
        hipLaunchKernelGGL(k_compact_pos, dim3(grid_for(n)), dim3(256), 0, st, n, flag, off,
                           c->act_pos.as<int32_t>());
    }
    // with every particle active the flags, their scan and the position list
    // are the identity: the grouping and the walk use sorted positions directly
    GroupCtx C{c->nd_link.as<int4>(), idx ? off : (const int32_t*)nullptr, c->sys_off.as<int64_t>(), c->n_sys,
               c->sys_levels, c->group_span, c->group_cap, c->group_split, c->group_pack};
    const int64_t* hdr = c->tree_hdr.as<int64_t>();
    int32_t* gcnt = c->grp_cnt.as<int32_t>();
    int32_t* goff = c->grp_off.as<int32_t>();
    hipLaunchKernelGGL(k_group_count, dim3(grid_for(c->max_nodes)), dim3(256), 0, st, C, hdr, c->max_nodes, gcnt);
    AG_TRY(ag_scan_i32(c, gcnt, goff, c->max_nodes));
    int32_t* ghdr = c->grp_hdr.as<int32_t>();
    hipLaunchKernelGGL(k_group_emit, dim3(grid_for(c->max_nodes)), dim3(256), 0, st, C, hdr, goff,
                       c->grp.as<int4>(), ghdr, ghdr + 8);
    *max_groups = mg;
    return AG_OK;
}

namespace {

// ---------------------------------------------------------------------------
// vector-charge moments of the adjoint weights
// ---------------------------------------------------------------------------
// per node (FP64, 31 doubles): W0 (3), W1 row-major (9: W1_bc = sum w_b y_c),
// W2 (18: for b = x, y, z the symmetric sum w_b y y^T as xx yy zz xy xz yz),
// number of charged particles; FP32 copy as 8 float4 (W0 + count, W1, W2).
constexpr int kW64 = 31;

__device__ void store_w(int64_t id, const double* r, double* __restrict__ w64, float4* __restrict__ wf) {
    double* o = w64 + id * kW64;
#pragma unroll
    for (int k = 0; k < kW64; ++k) o[k] = r[k];
    float4* f = wf + 8 * id;
    f[0] = make_float4((float)r[0], (float)r[1], (float)r[2], (float)r[30]);
#pragma unroll
    for (int q = 1; q < 8; ++q)
        f[q] = make_float4((float)r[4 * q - 1], (float)r[4 * q], (float)r[4 * q + 1],
                           q < 7 ? (float)r[4 * q + 2] : 0.f);
}

// sum_w w_b y_c y_e over the 6 symmetric (c, e) pairs into W2 (18 entries)
__device__ __forceinline__ void add_w2(double* W2, const double* wv, const double* y) {
    const int a[6] = {0, 1, 2, 0, 0, 1}, b[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int bb = 0; bb < 3; ++bb)
#pragma unroll
        for (int k = 0; k < 6; ++k) W2[6 * bb + k] += wv[bb] * y[a[k]] * y[b[k]];
}

// sorted weights: w of active rows, zero elsewhere
// weights in key order; a row carries its charge if it is listed: by the
// flags, or every row (all = 1), or none (all = 0 with no flags)
__global__ void k_gather_w(int64_t n, const int32_t* __restrict__ perm, const int32_t* __restrict__ flag, int all,
                           const double* __restrict__ w, double4* __restrict__ ws) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = perm[p];
        const bool charged = flag ? flag[p] != 0 : all != 0;
        ws[p] = charged ? make_double4(w[3 * i], w[3 * i + 1], w[3 * i + 2], 1.0) : make_double4(0, 0, 0, 0);
    }
}

__global__ void k_leaf_wmoments(const int64_t* __restrict__ hdr, const int32_t* __restrict__ leaves,
                                const int4* __restrict__ link, const double* __restrict__ m64,
                                const double4* __restrict__ spos, const double4* __restrict__ ws,
                                double* __restrict__ w64, float4* __restrict__ wf) {
    const int64_t nl = hdr[0] - hdr[2];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nl;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t id = leaves[t];
        const int4 L = link[id];
        const double* c = m64 + id * 25 + 1;   // node centre of mass
        double r[kW64];
#pragma unroll
        for (int q = 0; q < kW64; ++q) r[q] = 0.0;
        for (int j = L.y; j < L.y + L.z; ++j) {
            const double4 w = ws[j];
            if (w.w == 0.0) continue;
            const double4 x = spos[j];
            const double y[3] = {x.x - c[0], x.y - c[1], x.z - c[2]};
            const double wv[3] = {w.x, w.y, w.z};
            for (int b = 0; b < 3; ++b) {
                r[b] += wv[b];
                for (int cc = 0; cc < 3; ++cc) r[3 + 3 * b + cc] += wv[b] * y[cc];
            }
            add_w2(r + 12, wv, y);
            r[30] += 1.0;
        }
        store_w(id, r, w64, wf);
    }
}

// Shifted to the parent centre (y = y_child + dl):
//   W1_bc  = sum (W1_bc + W0_b dl_c)
//   W2_bce = sum (W2_bce + W1_bc dl_e + W1_be dl_c + W0_b dl_c dl_e)
// Levels l_hi down to l_lo: one level per launch (l_hi = l_lo, any grid),
// or several in a single-workgroup launch, the workgroup barrier between
// levels ordering each level after its children's.
__global__ void k_inner_wlevel(int l_hi, int l_lo, const int32_t* __restrict__ lvl,
                               const int32_t* __restrict__ lvl_list, const int4* __restrict__ child,
                               const double* __restrict__ m64, double* __restrict__ w64, float4* __restrict__ wf) {
  for (int level = l_hi; level >= l_lo; --level) {
    if (level < l_hi) __syncthreads();   // single-workgroup launches only
    const int t_lo = lvl[kLvlOff + level], t_hi = lvl[kLvlOff + level + 1];
    for (int64_t t = t_lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < t_hi;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int id = lvl_list[t];   // a level's nodes and their child rows share slots
        const int4 c0 = child[2 * t], c1 = child[2 * t + 1];
        const int ch8[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
        const double* c = m64 + (int64_t)id * 25 + 1;
        double r[kW64];
#pragma unroll
        for (int q = 0; q < kW64; ++q) r[q] = 0.0;
        for (int k8 = 0; k8 < 8; ++k8) {
            const int ch = ch8[k8];
            if (ch < 0) continue;
            const double* cw = w64 + (int64_t)ch * kW64;
            const double* cc = m64 + (int64_t)ch * 25 + 1;
            const double dl[3] = {cc[0] - c[0], cc[1] - c[1], cc[2] - c[2]};
            const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
            for (int b = 0; b < 3; ++b) {
                r[b] += cw[b];
                for (int q = 0; q < 3; ++q) r[3 + 3 * b + q] += cw[3 + 3 * b + q] + cw[b] * dl[q];
                for (int k = 0; k < 6; ++k) {
                    const int cc1 = ia[k], ee = ib[k];
                    r[12 + 6 * b + k] += cw[12 + 6 * b + k] + cw[3 + 3 * b + cc1] * dl[ee] +
                                         cw[3 + 3 * b + ee] * dl[cc1] + cw[b] * dl[cc1] * dl[ee];
                }
            }
            r[30] += cw[30];
        }
        store_w(id, r, w64, wf);
    }
  }
}

}  // namespace

static Tree make_tree(ag_ctx* c) {
    Tree T;
    T.com = c->nd_com.as<double4>();
    T.sh = c->tree_soft ? c->soft_s.as<float>() : nullptr;
    T.lo = c->nd_lo.as<float4>();
    T.hi = c->nd_hi.as<float4>();
    T.link = c->nd_link.as<int4>();
    T.mp = c->nd_mp.as<float4>();
    T.spos = c->spos.as<double4>();
    T.svf = c->svf.as<float4>();
    T.perm = c->perm.as<int32_t>();
    T.sys_root = c->sys_root.as<int32_t>();
    T.ws = c->wsorted.as<double4>();
    T.wf = c->nd_wf.as<float4>();
    return T;
}

static int walk_grid(ag_ctx* c, int64_t max_groups) {
    int dev_cus = 256;
    (void)hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device);
    int64_t blocks = (int64_t)dev_cus * c->walk_waves_per_cu;
    if (blocks > max_groups) blocks = (max_groups + 7) / 8 * 8;
    if (blocks < 8) blocks = 8;
    return (int)blocks;
}

// Ewald table: spacing box / 64 over the octant [0, box / 2]^3 of the cell
constexpr int kEwaldPerBox = 64;
constexpr int kEwaldNE = 32;
constexpr int kEwaldGroupDiv = 32;    // groups of half extent <= box / 32 sum once

static int ewald_table(ag_ctx* c) {
    if (c->ewald_tab_box == c->box && c->ewald_tab.bytes) return AG_OK;
    const int np = (kEwaldNE + 1) * (kEwaldNE + 1) * (kEwaldNE + 1);
    AG_TRY(ag_ensure(c, c->ewald_tab, (size_t)np * 5 * sizeof(float4)));
    hipLaunchKernelGGL(k_ewald_table, dim3((np + 127) / 128), dim3(128), 0, c->stream, c->box, kEwaldNE,
                       c->box / kEwaldPerBox, c->ewald_tab.as<float4>());
    c->ewald_tab_box = c->box;
    return AG_OK;
}

static WalkOut make_out(ag_ctx* c, double G) {
    WalkOut O{};
    O.stats = c->stats.as<unsigned long long>();
    O.G = G;
    O.flags = c->dflags.as<int32_t>();
    O.iter_cap = c->max_nodes + c->n + 1024;
    O.knn_scale = 1.0;
    O.small_node = c->small_node;
    O.mac_offset = c->mac_offset != 0;
    O.box = c->box;
    O.box_inv = c->box > 0.0 ? 1.0 / c->box : 0.0;
    O.boxf = (float)O.box;
    O.boxf_inv = (float)O.box_inv;
    // a margin of a few float ulps keeps every accepted node clear of the cut
    O.box_half = (float)(0.5 * c->box * (1.0 - 1e-5));
    O.ewald_theta = 1.0f / (float)c->ewald_open;
    O.ewald_grp = (float)(c->box / kEwaldGroupDiv);
    O.etab = c->ewald_tab.as<float4>();
    O.etab_ne = kEwaldNE;
    O.etab_h = (float)(c->box / kEwaldPerBox);
    O.etab_hinv = (float)(kEwaldPerBox / c->box);
    O.etab_range = (float)(c->box * kEwaldNE / kEwaldPerBox * (1.0 + 1e-4));   // a few ulps of slack
    return O;
}

// distance of every particle to its k-th nearest other particle, by a walk
// that opens every node and prunes by distance
int ag_launch_knn(ag_ctx* c, int32_t k, double scale, double* h_out) {
    int64_t mg = 0;
    AG_TRY(ag_prepare_groups(c, nullptr, c->n, &mg, nullptr, nullptr));
    Groups Gr{nullptr, c->grp.as<int4>(), c->grp_hdr.as<int32_t>()};
    WalkOut O = make_out(c, 1.0);
    O.stats = nullptr;
    O.knn_out = h_out;
    O.knn_scale = scale;
    O.knn_k = k;
    O.knn_n = c->n;
    O.box = c->tree_box;   // nearest images in the box the tree was built in
    PhaseScope phase(c, AG_PHASE_NEIGHBOUR);
    const unsigned grid = (unsigned)walk_grid(c, mg);
    int32_t* qctr = c->grp_hdr.as<int32_t>() + 8;
    const Tree T = make_tree(c);
    hipStream_t st = c->stream;
#define AG_KNN(CAP, PER) \
    hipLaunchKernelGGL((k_walk<KnnPolicy<CAP>, PER>), dim3(grid), dim3(kW), 0, st, T, Gr, O, qctr, 0.f, 0.f, 0.f, 0.f)
    const bool per = c->tree_box > 0.0;
    if (k <= 16) {
        if (per) AG_KNN(16, kNear); else AG_KNN(16, kOpen);
    } else if (k <= 32) {
        if (per) AG_KNN(32, kNear); else AG_KNN(32, kOpen);
    } else {
        if (per) AG_KNN(64, kNear); else AG_KNN(64, kOpen);
    }
#undef AG_KNN
    return AG_OK;
}

// Price & Monaghan lengths and Omega: the 64-neighbour walk in density mode
// (step 0), then the sum walk's Newton steps for the lengths the list
// cannot reach (step > 0; each launch re-arms the walk's work queues), run
// over the n_left rows the list pass left, grouped on their own)
int ag_launch_pm_lengths(ag_ctx* c, double n_ngb, double* h, double* omega, int step, int64_t n_left) {
    int64_t mg = 0;
    int32_t* left = reinterpret_cast<int32_t*>(reinterpret_cast<int*>(c->pm_brk.as<double>() + 3 * c->n) + kPmSteps);
    AG_TRY(ag_prepare_groups(c, step == 0 ? nullptr : left, step == 0 ? c->n : n_left, &mg, nullptr, nullptr));
    Groups Gr{c->all_active ? (const int32_t*)nullptr : c->act_pos.as<int32_t>(), c->grp.as<int4>(),
              c->grp_hdr.as<int32_t>()};
    WalkOut O = make_out(c, 1.0);
    O.stats = nullptr;
    O.knn_out = h;
    O.knn_k = c->n - 1 < 64 ? (int)(c->n - 1) : 64;
    O.knn_n = c->n;
    O.pm_ngb = n_ngb;
    O.pm_omega = omega;
    O.pm_lo = c->pm_brk.as<double>();
    O.pm_hi = O.pm_lo + c->n;
    O.pm_cur = O.pm_hi + c->n;
    O.pm_active = reinterpret_cast<int*>(O.pm_cur + c->n) + step;
    O.pm_idx = left;
    // every particle lies within the root's diagonal D of every other, so
    // at h = D / u* the sum is at least n (1 - 6 u*^2) >= 3 N / 32 (w(u) >=
    // 1 - 6 u^2 for u < 1/2)
    const double f = 3.0 * n_ngb / 32.0 / (double)c->n;
    const double us = std::min(0.5, std::sqrt((1.0 - f) / 6.0));
    O.pm_hiscale = 1.01 / us;
    PhaseScope phase(c, AG_PHASE_NEIGHBOUR);
    const unsigned grid = (unsigned)walk_grid(c, mg);
    int32_t* qctr = c->grp_hdr.as<int32_t>() + 8;
    if (step == 0) {
        hipLaunchKernelGGL((k_walk<KnnPolicy<64, true>, kOpen>), dim3(grid), dim3(kW), 0, c->stream, make_tree(c), Gr,
                           O, qctr, 0.f, 0.f, 0.f, 0.f);
    } else {
        hipLaunchKernelGGL((k_walk<PmPolicy<2>, kOpen>), dim3(grid), dim3(kW), 0, c->stream, make_tree(c), Gr, O,
                           qctr, 0.f, 0.f, 0.f, 0.f);
    }
    return AG_OK;
}

// Price & Monaghan sums: Z (mode 0, z_out) or the correction (mode 1, acc)
int ag_launch_pm_sum(ag_ctx* c, int mode, double n_ngb, double G, const double* omega, const double* z,
                     double* z_out, double* acc, const int32_t* idx, const int64_t* n_dev, bool add) {
    int64_t mg = 0;
    AG_TRY(ag_prepare_groups(c, idx, c->n, &mg, idx ? n_dev : nullptr, nullptr));
    Groups Gr{c->all_active ? (const int32_t*)nullptr : c->act_pos.as<int32_t>(), c->grp.as<int4>(),
              c->grp_hdr.as<int32_t>()};
    WalkOut O = make_out(c, G);
    O.stats = nullptr;
    O.pm_ngb = n_ngb;
    O.pm_G = G;
    O.pm_h = c->soft_h.as<double>();
    O.pm_om = omega;
    O.pm_z = z;
    O.pm_zout = z_out;
    O.pm_acc = acc;
    O.pm_add = add || idx != nullptr;
    PhaseScope phase(c, AG_PHASE_NEIGHBOUR);
    const unsigned grid = (unsigned)walk_grid(c, mg);
    const Tree T = make_tree(c);
    int32_t* qctr = c->grp_hdr.as<int32_t>() + 8;
    if (mode == 0)
        hipLaunchKernelGGL((k_walk<PmPolicy<0>, kOpen>), dim3(grid), dim3(kW), 0, c->stream, T, Gr, O, qctr, 0.f, 0.f,
                           0.f, 0.f);
    else
        hipLaunchKernelGGL((k_walk<PmPolicy<1>, kOpen>), dim3(grid), dim3(kW), 0, c->stream, T, Gr, O, qctr, 0.f, 0.f,
                           0.f, 0.f);
    return AG_OK;
}

int ag_launch_eval(ag_ctx* c, const int32_t* idx, int64_t n_act, double theta, double eps, double G, double* acc,
                   double* jerk, double* tidal, const int64_t* n_dev, int64_t* n_total) {
    int64_t mg = 0;
    AG_TRY(ag_prepare_groups(c, idx, n_act, &mg, n_dev, n_total));
    Groups Gr{c->all_active ? (const int32_t*)nullptr : c->act_pos.as<int32_t>(), c->grp.as<int4>(),
              c->grp_hdr.as<int32_t>()};
    const bool ewald = c->box > 0.0 && c->ewald;
    if (ewald) AG_TRY(ewald_table(c));
    WalkOut O = make_out(c, G);   // after the table, for its address
    O.acc = acc;
    O.jerk = jerk;
    O.tidal = tidal;
    if (c->rel_n > 0) {
        O.rel_a = c->rel_a.as<float>();
        O.rel_alpha = (float)c->rel_alpha;
        O.rel_g = (float)fabs(G);
    }
    const float th = (float)theta;
    const float e2 = (float)(eps * eps);
    const unsigned grid = (unsigned)walk_grid(c, mg);
    int32_t* qctr = c->grp_hdr.as<int32_t>() + 8;
    {
        PhaseScope phase(c, AG_PHASE_WALK);
        const Tree T = make_tree(c);
        const float h2 = e2, hi = (float)(1.0 / eps);
        hipStream_t st = c->stream;
        if (c->tree_soft) {   // per-particle softening lengths
            if (ewald)
                hipLaunchKernelGGL((k_walk<ForwardPolicy, kEwald, true>), dim3(grid), dim3(kW), 0, st, T, Gr, O, qctr,
                                   th * th, e2, h2, hi);
            else if (c->box > 0.0)
                hipLaunchKernelGGL((k_walk<ForwardPolicy, kNear, true>), dim3(grid), dim3(kW), 0, st, T, Gr, O, qctr,
                                   th * th, e2, h2, hi);
            else
                hipLaunchKernelGGL((k_walk<ForwardPolicy, kOpen, true>), dim3(grid), dim3(kW), 0, st, T, Gr, O, qctr,
                                   th * th, e2, h2, hi);
        } else if (ewald) {
            hipLaunchKernelGGL((k_walk<ForwardPolicy, kEwald>), dim3(grid), dim3(kW), 0, st, T, Gr, O, qctr, th * th,
                               e2, h2, hi);
        } else if (c->box > 0.0) {
            hipLaunchKernelGGL((k_walk<ForwardPolicy, kNear>), dim3(grid), dim3(kW), 0, st, T, Gr, O, qctr, th * th,
                               e2, h2, hi);
        } else {
            hipLaunchKernelGGL((k_walk<ForwardPolicy, kOpen>), dim3(grid), dim3(kW), 0, st, T, Gr, O, qctr, th * th,
                               e2, h2, hi);
        }
    }
    if (ewald && (acc || tidal)) {
        // what the periodic images add to g and T, at the same images
        AG_TRY(ag_ensure(c, c->ewald_q, 8 * sizeof(int32_t)));
        PhaseScope phase(c, AG_PHASE_EWALD);
        hipLaunchKernelGGL(k_fill0, dim3(1), dim3(64), 0, c->stream, c->ewald_q.as<int32_t>(), (int64_t)8);
        WalkOut E = O;
        E.stats = nullptr;
        E.rel_a = nullptr;
        hipLaunchKernelGGL((k_walk<EwaldPolicy, kEwald>), dim3(grid), dim3(kW), 0, c->stream, make_tree(c), Gr, E,
                           c->ewald_q.as<int32_t>(), 0.f, 0.f, e2, (float)(1.0 / eps));
    }
    return AG_OK;
}

// Adjoint of L = sum_k w_k . g_k:
//   1. forward walk for T at the listed rows (the T_k w_k term);
//   2. sorted weights (zero on unlisted rows) and their node moments W0, W1, W2;
//   3. adjoint walk over all n targets with the same opening test, both walks
//      at theta * AG_OPT_ADJOINT_OPEN / 100.
int ag_launch_backward(ag_ctx* c, const int32_t* idx, int64_t n_act, const double* w, double theta, double eps,
                       double G, double* dLdx, double* dLdm) {
    const int64_t n = c->n;
    AG_TRY(ag_ensure(c, c->tmp_tidal, n * 6 * sizeof(double)));
    AG_TRY(ag_ensure(c, c->wsorted, n * sizeof(double4)));
    AG_TRY(ag_ensure(c, c->nd_w, c->max_nodes * kW64 * sizeof(double)));
    AG_TRY(ag_ensure(c, c->nd_wf, c->max_nodes * 8 * sizeof(float4)));
    double* tin = c->tmp_tidal.as<double>();
    // both walks open nodes at a fraction of theta: their kernels (the tidal
    // tensor and J, 1/r^3) are one derivative deeper than the force's
    theta *= c->adj_open / 100.0;
    if (n_act > 0) AG_TRY(ag_launch_eval(c, idx, n_act, theta, eps, G, nullptr, nullptr, tin));
    // charges: the listed rows (flags of that evaluation), all rows, or none
    const int32_t* cflag = (n_act > 0 && !c->all_active) ? c->act_flag.as<int32_t>() : nullptr;
    const int call = n_act > 0 && c->all_active ? 1 : 0;

    PhaseScope phase(c, AG_PHASE_ADJOINT);
    hipStream_t st = c->stream;
    hipLaunchKernelGGL(k_gather_w, dim3(grid_for(n)), dim3(256), 0, st, n, c->perm.as<int32_t>(), cflag, call, w,
                       c->wsorted.as<double4>());
    hipLaunchKernelGGL(k_leaf_wmoments, dim3(grid_for(n / 4 + 1)), dim3(256), 0, st, c->tree_hdr.as<int64_t>(),
                       c->leaf_list.as<int32_t>(), c->nd_link.as<int4>(), c->nd_64.as<double>(),
                       c->spos.as<double4>(), c->wsorted.as<double4>(), c->nd_w.as<double>(), c->nd_wf.as<float4>());
    const int64_t inner_bound = c->max_nodes - n;
    int g = grid_for(inner_bound > 0 ? inner_bound : 1);
    if (g > 128) g = 128;
    {
        // levels below the deepest the host has seen in one single-workgroup
        // launch (usually empty), then one launch per level down to 3, and
        // levels 2-0 (at most 73 nodes) in one single-workgroup launch
        const int32_t* lvl = reinterpret_cast<const int32_t*>(c->tree_hdr.as<int64_t>() + 8);
        const int32_t* ll = c->lvl_list.as<int32_t>();
        const int4* ch = c->child.as<int4>();
        const double* m64 = c->nd_64.as<double>();
        double* w64 = c->nd_w.as<double>();
        float4* wf = c->nd_wf.as<float4>();
        constexpr int kTop = 2;
        int lc = c->seen_max_level - 1;
        if (c->seen_max_level < 0 || lc > AG_MAX_LEVEL - 1) lc = AG_MAX_LEVEL - 1;
        if (lc < kTop + 1) lc = kTop;
        if (lc < AG_MAX_LEVEL - 1)
            hipLaunchKernelGGL(k_inner_wlevel, dim3(1), dim3(256), 0, st, AG_MAX_LEVEL - 1, lc + 1, lvl, ll, ch, m64,
                               w64, wf);
        for (int l = lc; l > kTop; --l)
            hipLaunchKernelGGL(k_inner_wlevel, dim3(g), dim3(256), 0, st, l, l, lvl, ll, ch, m64, w64, wf);
        hipLaunchKernelGGL(k_inner_wlevel, dim3(1), dim3(256), 0, st, kTop, 0, lvl, ll, ch, m64, w64, wf);
    }
    int64_t mg = 0;
    AG_TRY(ag_prepare_groups(c, nullptr, n, &mg, nullptr, nullptr));   // every particle is a target
    Groups Gr{c->all_active ? (const int32_t*)nullptr : c->act_pos.as<int32_t>(), c->grp.as<int4>(),
              c->grp_hdr.as<int32_t>()};
    WalkOut O = make_out(c, G);
    O.dldx = dLdx;
    O.dldm = dLdm;
    O.tin = tin;
    const float th = (float)theta;
    const float e2 = (float)(eps * eps);
    hipLaunchKernelGGL((k_walk<AdjointPolicy, kOpen>), dim3((unsigned)walk_grid(c, mg)), dim3(kW), 0, st,
                       make_tree(c), Gr,
                       O, c->grp_hdr.as<int32_t>() + 8, th * th, e2, e2, (float)(1.0 / eps));
    return AG_OK;
}
