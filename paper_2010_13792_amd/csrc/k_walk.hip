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
    double box, box_inv;        // periodic cube side and inverse (periodic walks only)
    float boxf, boxf_inv, box_half;
    double* dldx;       // adjoint outputs
    double* dldm;
    const double* tin;  // adjoint: tidal tensor rows of the charged targets
};

// group geometry shared by every lane (uniform values)
struct GroupBox {
    double cx, cy, cz;          // centre (FP64)
    float hx, hy, hz;           // half extents (rounded up)
    float lox, loy, loz, hix, hiy, hiz;   // absolute box, rounded outward
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
// Periodic (kPer): distances are taken at the nearest image of the node, and
// a node is accepted only if, along every axis, all of its box lies within
// half a box side of all of the group box -- then every particle-target pair
// of the node has that same nearest image, and the multipole stands for it.
template <bool kPer>
__device__ __forceinline__ bool mac_accept(const GroupBox& g, const double4 c, const float4 lo, const float4 hi,
                                           float theta2, float eps2, bool offset, const WalkOut& O) {
    double cdx = c.x - g.cx, cdy = c.y - g.cy, cdz = c.z - g.cz;
    if (kPer) {
        cdx = near_img(cdx, O);
        cdy = near_img(cdy, O);
        cdz = near_img(cdz, O);
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
    if (!kPer) {
        gx = fmaxf(fmaxf(lo.x - g.hix, g.lox - hi.x), 0.f);
        gy = fmaxf(fmaxf(lo.y - g.hiy, g.loy - hi.y), 0.f);
        gz = fmaxf(fmaxf(lo.z - g.hiz, g.loz - hi.z), 0.f);
    } else {
        // box centre offset at its nearest image, and the half extents
        const float bx = fabsf((float)near_img(0.5 * ((double)lo.x + (double)hi.x) - g.cx, O));
        const float by = fabsf((float)near_img(0.5 * ((double)lo.y + (double)hi.y) - g.cy, O));
        const float bz = fabsf((float)near_img(0.5 * ((double)lo.z + (double)hi.z) - g.cz, O));
        const float ex = 0.5f * (hi.x - lo.x) + g.hx;
        const float ey = 0.5f * (hi.y - lo.y) + g.hy;
        const float ez = 0.5f * (hi.z - lo.z) + g.hz;
        if (bx + ex >= O.box_half || by + ey >= O.box_half || bz + ez >= O.box_half) return false;
        gx = fmaxf(bx - ex, 0.f);
        gy = fmaxf(by - ey, 0.f);
        gz = fmaxf(bz - ez, 0.f);
    }
    const float sep2 = gx * gx + gy * gy + gz * gz;
    return r2 > 0.f && L * L <= theta2 * r2 && sep2 >= eps2;
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
};

// ---- forward: g, j and S = -T from particle masses and node multipoles ----
struct ForwardPolicy {
    static constexpr bool kSkipEmpty = false;
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
    template <bool kPer>
    __device__ static void stage_particle(Lds& S, const Tree& T, const GroupBox& gb, int lane, int pk,
                                          const WalkOut& O) {
        const double4 q = T.spos[pk];
        const float4 u = T.svf[pk];
        double dx = q.x - gb.cx, dy = q.y - gb.cy, dz = q.z - gb.cz;
        if (kPer) {
            dx = near_img(dx, O);
            dy = near_img(dy, O);
            dz = near_img(dz, O);
        }
        S.tile[lane] = make_float4((float)dx, (float)dy, (float)dz, u.w);
        S.tile[kW + lane] = u;
        S.tidx[lane] = pk;
    }
    // The quantities of pair_interact, written as multiply-add chains into
    // the accumulators, with the m f I part of S summed once per tile.  The
    // self pair has d = 0 exactly (both sides round the same FP64 position),
    // so it always takes the softened branch, where it is dropped.  Periodic:
    // each pair is taken at its own nearest image.
    template <bool kPer>
    __device__ static void particles(const Lds& S, int cnt, const Target& t, Acc& acc, float h2, float hinv,
                                     int k0, int ks, const WalkOut& O) {
        PairAcc<float> F;
        F.zero();
        float smf = 0.f;
        for (int k = k0; k < cnt; k += ks) {
            const float4 q = S.tile[k];
            const float4 u = S.tile[kW + k];
            float dx = q.x - t.tx, dy = q.y - t.ty, dz = q.z - t.tz;
            if (kPer) {
                dx = near_imgf(dx, O);
                dy = near_imgf(dy, O);
                dz = near_imgf(dz, O);
            }
            const float nx = u.x - t.vx, ny = u.y - t.vy, nz = u.z - t.vz;
            const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
            float mf, mD;
            if (r2 >= h2) {
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float ri2 = ri * ri;
                mf = q.w * (ri * ri2);
                mD = -3.f * mf * ri2;
            } else {
                float f, D;
                spline_fd<float>(r2, hinv, f, D);
                const float mj = (S.tidx[k] == t.p) ? 0.f : q.w;
                mf = mj * f;
                mD = mj * D;
            }
            F.ax = __builtin_fmaf(mf, dx, F.ax);
            F.ay = __builtin_fmaf(mf, dy, F.ay);
            F.az = __builtin_fmaf(mf, dz, F.az);
            const float sd = mD * __builtin_fmaf(dz, nz, __builtin_fmaf(dy, ny, dx * nx));
            F.jx = __builtin_fmaf(sd, dx, __builtin_fmaf(mf, nx, F.jx));
            F.jy = __builtin_fmaf(sd, dy, __builtin_fmaf(mf, ny, F.jy));
            F.jz = __builtin_fmaf(sd, dz, __builtin_fmaf(mf, nz, F.jz));
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
    template <bool kPer>
    __device__ static void stage_node(Lds& S, const Tree& T, const GroupBox& gb, int lane, int nk,
                                      const WalkOut& O) {
        const double4 c = T.com[nk];
        const float4 m0 = T.mp[4 * nk], m1 = T.mp[4 * nk + 1], m2 = T.mp[4 * nk + 2], m3 = T.mp[4 * nk + 3];
        float4* d = S.tile;
        double dx = c.x - gb.cx, dy = c.y - gb.cy, dz = c.z - gb.cz;
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
    __device__ static void nodes(const Lds& S, int cnt, const Target& t, Acc& acc, int k0, int ks) {
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
    __device__ static void finish(const Tree& T, const WalkOut& O, const Acc& A, int p) {
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
    using Lds = WalkLds<9>;
    struct Acc {
        double vx, vy, vz, s;
        __device__ void zero() { vx = vy = vz = s = 0.0; }
        __device__ void add(const Acc& o) { vx += o.vx; vy += o.vy; vz += o.vz; s += o.s; }
    };
    template <bool kPer>
    __device__ static void stage_particle(Lds& S, const Tree& T, const GroupBox& gb, int lane, int pk,
                                          const WalkOut&) {
        static_assert(!kPer, "the adjoint walk has no periodic form");
        const double4 q = T.spos[pk];
        const double4 w = T.ws[pk];
        S.tile[lane] = make_float4((float)(q.x - gb.cx), (float)(q.y - gb.cy), (float)(q.z - gb.cz), 0.f);
        S.tile[kW + lane] = make_float4((float)w.x, (float)w.y, (float)w.z, 0.f);
        S.tidx[lane] = pk;
    }
    template <bool kPer>
    __device__ static void particles(const Lds& S, int cnt, const Target& t, Acc& acc, float h2, float hinv,
                                     int k0, int ks, const WalkOut&) {
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
    template <bool kPer>
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
    __device__ static void nodes(const Lds& S, int cnt, const Target& t, Acc& acc, int k0, int ks) {
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
    __device__ static void finish(const Tree& T, const WalkOut& O, const Acc& A, int p) {
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
template <class Pol, bool kPer>
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
    const GroupBox gb = group_box(xi.x, xi.y, xi.z);
    Target tg;
    tg.tx = (float)(xi.x - gb.cx);
    tg.ty = (float)(xi.y - gb.cy);
    tg.tz = (float)(xi.z - gb.cz);
    tg.vx = vi.x;
    tg.vy = vi.y;
    tg.vz = vi.z;
    tg.p = p_i;

    typename Pol::Acc acc;
    acc.zero();
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
        Pol::template particles<kPer>(S, cnt, tg, acc, h2, hinv, part, sub, O);
        n_pp += (uint64_t)cnt;
        __syncthreads();
    };
    auto flush_nodes = [&](int base, int cnt) {
        if (lane < cnt) Pol::template stage_node<kPer>(S, T, gb, lane, S.nlist[base + lane], O);
        __syncthreads();
        Pol::nodes(S, cnt, tg, acc, part, sub);
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
            if (Pol::kSkipEmpty && T.wf[8 * a].w == 0.f) {
                ca = L.x;                  // no charge below this node
            } else {
                const bool acc_ok =
                    mac_accept<kPer>(gb, T.com[a], T.lo[a], T.hi[a], theta2, eps2, O.mac_offset, O);
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

    if (sub > 1) {
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
    if (part == 0) Pol::finish(T, O, acc, p_i);
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
template <class Pol, bool kPer>
__global__ void __launch_bounds__(kW, 4) k_walk(Tree T, Groups Gr, WalkOut O, int* __restrict__ qctr,
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
        walk_group<Pol, kPer>(S, T, Gr, O, Gr.grp[g], theta2, eps2, h2, hinv);
        __syncthreads();
    }
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
__global__ void k_mark_stamp(int64_t n_act, const int32_t* __restrict__ idx, int64_t n,
                             const int32_t* __restrict__ rank, int32_t* __restrict__ stamp,
                             int32_t* __restrict__ flags) {
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

__global__ void k_mark_check(int64_t n_act, const int32_t* __restrict__ idx, int64_t n,
                             const int32_t* __restrict__ rank, const int32_t* __restrict__ stamp,
                             int32_t* __restrict__ flag, int32_t* __restrict__ flags) {
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
    auto emit = [&](int start, int cnt, int64_t pos) {
        if (out) out[ng] = make_int4(start, cnt, C.n_sys > 1 ? sys_of_pos(C, pos) : 0, 0);
        ++ng;
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
    for (int ch = id + 1, k8 = 0; ch < L.x && k8 < 8; ch = C.link[ch].x, ++k8) {
        const int4 Lc = C.link[ch];
        const int c0 = C.aoff ? C.aoff[Lc.y] : Lc.y;
        const int ac = (C.aoff ? C.aoff[Lc.y + Lc.z] : Lc.y + Lc.z) - c0;
        const bool leafc = (Lc.w & 0x100) != 0;
        const bool bigc = (Lc.w & 0xff) < C.sys_levels || ac > C.cap || (C.span > 0 && !leafc && Lc.z > C.span);
        if (bigc || ac == 0 || forced) {
            if (run_cnt > 0) emit(run_start, run_cnt, run_pos);
            run_cnt = 0;
            run_span = 0;
            if (forced && !bigc && ac > 0) emit(c0, ac, Lc.y);
            continue;
        }
        if (run_cnt + ac > C.cap || (C.span > 0 && run_span + Lc.z > C.span)) {
            if (run_cnt > 0) emit(run_start, run_cnt, run_pos);
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
    if (run_cnt > 0) emit(run_start, run_cnt, run_pos);
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

int ag_prepare_groups(ag_ctx* c, const int32_t* idx, int64_t n_act, int64_t* max_groups) {
    const int64_t n = c->n;
    const int64_t mg = n_act + c->n_sys + 1;   // every group holds at least one target
    AG_TRY(ag_ensure(c->act_flag, n * 4));
    AG_TRY(ag_ensure(c->act_off, (n + 1) * 4));
    AG_TRY(ag_ensure(c->act_pos, n * 4));
    AG_TRY(ag_ensure(c->grp, mg * 16));
    AG_TRY(ag_ensure(c->grp_hdr, (16 + AG_MAX_SYS + 1) * 4));
    AG_TRY(ag_ensure(c->grp_cnt, (c->max_nodes + 1) * 4));
    AG_TRY(ag_ensure(c->grp_off, (c->max_nodes + 1) * 4));
    PhaseScope phase(c, AG_PHASE_GROUPS);
    hipStream_t st = c->stream;
    int32_t* flag = c->act_flag.as<int32_t>();
    int32_t* off = c->act_off.as<int32_t>();
    c->all_active = idx == nullptr;
    if (idx) {
        hipLaunchKernelGGL(k_fill0, dim3(grid_for(n)), dim3(256), 0, st, flag, n);
        // the scan output doubles as the stamp array until the scan runs
        hipLaunchKernelGGL(k_mark_stamp, dim3(grid_for(n_act)), dim3(256), 0, st, n_act, idx, n,
                           c->rank.as<int32_t>(), off, c->dflags.as<int32_t>());
        hipLaunchKernelGGL(k_mark_check, dim3(grid_for(n_act)), dim3(256), 0, st, n_act, idx, n,
                           c->rank.as<int32_t>(), off, flag, c->dflags.as<int32_t>());
        AG_TRY(ag_scan_i32(c, flag, off, n));
        hipLaunchKernelGGL(k_compact_pos, dim3(grid_for(n)), dim3(256), 0, st, n, flag, off,
                           c->act_pos.as<int32_t>());
    }
    // with every particle active the flags, their scan and the position list
    // are the identity: the grouping and the walk use sorted positions directly
    GroupCtx C{c->nd_link.as<int4>(), idx ? off : (const int32_t*)nullptr, c->sys_off.as<int64_t>(), c->n_sys,
               c->sys_levels, c->group_span, c->group_cap};
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
__global__ void k_inner_wlevel(int level, const int32_t* __restrict__ lvl, const int32_t* __restrict__ lvl_list,
                               const int32_t* __restrict__ ilist, const int4* __restrict__ child,
                               const double* __restrict__ m64, double* __restrict__ w64, float4* __restrict__ wf) {
    const int t_lo = lvl[kLvlOff + level], t_hi = lvl[kLvlOff + level + 1];
    for (int64_t t = t_lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < t_hi;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int in = lvl_list[t];
        const int id = ilist[in];
        const int4 c0 = child[2 * in], c1 = child[2 * in + 1];
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

}  // namespace

static Tree make_tree(ag_ctx* c) {
    Tree T;
    T.com = c->nd_com.as<double4>();
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

static WalkOut make_out(ag_ctx* c, double G) {
    WalkOut O{};
    O.stats = c->stats.as<unsigned long long>();
    O.G = G;
    O.flags = c->dflags.as<int32_t>();
    O.iter_cap = c->max_nodes + c->n + 1024;
    O.small_node = c->small_node;
    O.mac_offset = c->mac_offset != 0;
    O.box = c->box;
    O.box_inv = c->box > 0.0 ? 1.0 / c->box : 0.0;
    O.boxf = (float)O.box;
    O.boxf_inv = (float)O.box_inv;
    // a margin of a few float ulps keeps every accepted node clear of the cut
    O.box_half = (float)(0.5 * c->box * (1.0 - 1e-5));
    return O;
}

int ag_launch_eval(ag_ctx* c, const int32_t* idx, int64_t n_act, double theta, double eps, double G, double* acc,
                   double* jerk, double* tidal) {
    int64_t mg = 0;
    AG_TRY(ag_prepare_groups(c, idx, n_act, &mg));
    Groups Gr{c->all_active ? (const int32_t*)nullptr : c->act_pos.as<int32_t>(), c->grp.as<int4>(),
              c->grp_hdr.as<int32_t>()};
    WalkOut O = make_out(c, G);
    O.acc = acc;
    O.jerk = jerk;
    O.tidal = tidal;
    const float th = (float)theta;
    const float e2 = (float)(eps * eps);
    {
        PhaseScope phase(c, AG_PHASE_WALK);
        if (c->box > 0.0)
            hipLaunchKernelGGL((k_walk<ForwardPolicy, true>), dim3((unsigned)walk_grid(c, mg)), dim3(kW), 0,
                               c->stream, make_tree(c), Gr, O, c->grp_hdr.as<int32_t>() + 8, th * th, e2, e2,
                               (float)(1.0 / eps));
        else
            hipLaunchKernelGGL((k_walk<ForwardPolicy, false>), dim3((unsigned)walk_grid(c, mg)), dim3(kW), 0,
                               c->stream, make_tree(c), Gr, O, c->grp_hdr.as<int32_t>() + 8, th * th, e2, e2,
                               (float)(1.0 / eps));
    }
    return AG_OK;
}

// Adjoint of L = sum_k w_k . g_k:
//   1. forward walk for T at the listed rows (the T_k w_k term);
//   2. sorted weights (zero on unlisted rows) and their node moments W0, W1;
//   3. adjoint walk over all n targets with the same opening test.
int ag_launch_backward(ag_ctx* c, const int32_t* idx, int64_t n_act, const double* w, double theta, double eps,
                       double G, double* dLdx, double* dLdm) {
    const int64_t n = c->n;
    AG_TRY(ag_ensure(c->tmp_tidal, n * 6 * sizeof(double)));
    AG_TRY(ag_ensure(c->wsorted, n * sizeof(double4)));
    AG_TRY(ag_ensure(c->nd_w, c->max_nodes * kW64 * sizeof(double)));
    AG_TRY(ag_ensure(c->nd_wf, c->max_nodes * 8 * sizeof(float4)));
    double* tin = c->tmp_tidal.as<double>();
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
    for (int l = AG_MAX_LEVEL - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_inner_wlevel, dim3(g), dim3(256), 0, st, l,
                           reinterpret_cast<const int32_t*>(c->tree_hdr.as<int64_t>() + 8),
                           c->lvl_list.as<int32_t>(), c->in_list.as<int32_t>(), c->child.as<int4>(),
                           c->nd_64.as<double>(),
                           c->nd_w.as<double>(), c->nd_wf.as<float4>());
    int64_t mg = 0;
    AG_TRY(ag_prepare_groups(c, nullptr, n, &mg));   // every particle is a target
    Groups Gr{c->all_active ? (const int32_t*)nullptr : c->act_pos.as<int32_t>(), c->grp.as<int4>(),
              c->grp_hdr.as<int32_t>()};
    WalkOut O = make_out(c, G);
    O.dldx = dLdx;
    O.dldm = dLdm;
    O.tin = tin;
    const float th = (float)theta;
    const float e2 = (float)(eps * eps);
    hipLaunchKernelGGL((k_walk<AdjointPolicy, false>), dim3((unsigned)walk_grid(c, mg)), dim3(kW), 0, st,
                       make_tree(c), Gr,
                       O, c->grp_hdr.as<int32_t>() + 8, th * th, e2, e2, (float)(1.0 / eps));
    return AG_OK;
}
