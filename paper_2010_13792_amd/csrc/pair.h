// pair.h -- the softened pair interaction used by the direct sum and by the
// tree walk's particle-particle part.
//
// For a source of mass m at separation d = x_j - x_i moving with relative
// velocity nu = v_j - v_i the target gains
//     g += m f(r) d
//     j += m [ f(r) nu + D(r) (d.nu) d ]       (time derivative of m f d)
//     S += m [ f(r) I + D(r) d d^T ]           (the tidal tensor is T = -G S)
// with D = f'(r)/r.  f is the cubic-spline (M4) softened force factor of
// compact support h: f = mu(u)/r^3, u = r/h, mu the kernel mass inside r,
// written in the forms that stay finite at r = 0:
//     u < 1/2:    f = h^-3 (32/3 - 192/5 u^2 + 32 u^3),     D = h^-5 (96 u - 384/5)
//     1/2<=u<1:   f = h^-3 (64/3 - 48 u + 192/5 u^2 - 32/3 u^3 - 1/(15 u^3)),
//                 D = h^-5 (-48/u + 384/5 - 32 u + 1/(5 u^5))
//     u >= 1:     f = r^-3, D = -3 r^-5.
#pragma once
#include <hip/hip_runtime.h>

template <class R>
struct PairAcc {
    R ax, ay, az, jx, jy, jz, sxx, syy, szz, sxy, sxz, syz;
    __device__ __forceinline__ void zero() {
        ax = ay = az = jx = jy = jz = sxx = syy = szz = sxy = sxz = syz = R(0);
    }
};

__device__ __forceinline__ float ag_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double ag_rsqrt(double x) { return 1.0 / sqrt(x); }

// softened f and D for r2 < h^2 (the kernel interior)
template <class R>
__device__ __forceinline__ void spline_fd(R r2, R hinv, R& f, R& D) {
    const R r = sqrt(r2);
    const R u = r * hinv;
    const R h2i = hinv * hinv;
    const R h3 = h2i * hinv;
    const R h5 = h3 * h2i;
    if (u < R(0.5)) {
        f = h3 * (R(32.0 / 3.0) + u * u * (R(-192.0 / 5.0) + R(32.0) * u));
        D = h5 * (R(96.0) * u - R(384.0 / 5.0));
    } else {
        const R ui = R(1) / u;
        const R ui3 = ui * ui * ui;
        f = h3 * (R(64.0 / 3.0) + u * (R(-48.0) + u * (R(192.0 / 5.0) - R(32.0 / 3.0) * u))
                  - R(1.0 / 15.0) * ui3);
        D = h5 * (R(-48.0) * ui + R(384.0 / 5.0) - R(32.0) * u + R(0.2) * ui3 * ui * ui);
    }
}

template <class R>
__device__ __forceinline__ void pair_interact(R dx, R dy, R dz, R nx, R ny, R nz, R mj, R h2,
                                              R hinv, PairAcc<R>& A) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    R f, D;
    if (r2 >= h2) {
        const R ri = ag_rsqrt(r2);
        const R ri2 = ri * ri;
        f = ri * ri2;
        D = R(-3) * f * ri2;
    } else {
        spline_fd<R>(r2, hinv, f, D);
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

// the same pair term with a softening length per particle: f and D are the
// means of the two particles' kernels (each Newtonian beyond its own length)
template <class R>
__device__ __forceinline__ void pair_interact_soft(R dx, R dy, R dz, R nx, R ny, R nz, R mj, R hi_, R hj,
                                                   PairAcc<R>& A) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    R fs[2], Ds[2];
    const R hs[2] = {hi_, hj};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (r2 >= hs[k] * hs[k]) {
            const R ri = ag_rsqrt(r2);
            const R ri2 = ri * ri;
            fs[k] = ri * ri2;
            Ds[k] = R(-3) * fs[k] * ri2;
        } else {
            spline_fd<R>(r2, R(1) / hs[k], fs[k], Ds[k]);
        }
    }
    const R mf = mj * (R(0.5) * (fs[0] + fs[1]));
    const R mD = mj * (R(0.5) * (Ds[0] + Ds[1]));
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

