// Device-side arithmetic of one THIIM split-field update (gfx950).
//
// Every sweep variant (naive, fused, temporally blocked, adjoint helpers)
// calls update_h / update_e below, so all of them perform exactly the same
// sequence of IEEE operations per element and their results are
// bit-identical.  The file is compiled with -ffp-contract=off: the only fused
// multiply-adds are the explicit ones written here.
//
// Update form (Sec. I-A Eq. (3)/(4) solved for the new value; Listings 1/2):
//     F_new = t F_old [+ Src] + c d,   d = s * (difference of G along axis),
// with G the sum of the two split parts of the driving component, s the sign
// of that derivative in the curl, H using the backward difference
// G(p) - G(p - e) and E the forward difference G(p + e) - G(p) (Fig. 3: the
// two fields depend on each other in opposite directions).
#pragma once
#include <hip/hip_runtime.h>

namespace thiim {

// split components (listing naming F_ab: part of F_a driven by component b)
enum Comp { HXY = 0, HXZ, HYX, HYZ, HZX, HZY, EXY, EXZ, EYX, EYZ, EZX, EZY };
// coefficient arrays: t_q = q, c_q = 12 + q, Src of H_xy, H_yx, E_xy, E_yx
enum CoefIdx { SRC_HXY = 24, SRC_HYX = 25, SRC_EXY = 26, SRC_EYX = 27 };
constexpr int NCOMP = 12;
constexpr int NCOEF = 28;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b) {
    return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 czero() { return make_double2(0.0, 0.0); }

// t * f + src + c * d  (complex), fixed operation order
__device__ __forceinline__ double2 upd_src(double2 f, double2 t, double2 c,
                                           double2 d, double2 src) {
    double re = __fma_rn(t.x, f.x, src.x);
    re = __fma_rn(-t.y, f.y, re);
    re = __fma_rn(c.x, d.x, re);
    re = __fma_rn(-c.y, d.y, re);
    double im = __fma_rn(t.x, f.y, src.y);
    im = __fma_rn(t.y, f.x, im);
    im = __fma_rn(c.x, d.y, im);
    im = __fma_rn(c.y, d.x, im);
    return make_double2(re, im);
}

// t * f + c * d  (complex), fixed operation order
__device__ __forceinline__ double2 upd(double2 f, double2 t, double2 c,
                                       double2 d) {
    double re = t.x * f.x;
    re = __fma_rn(-t.y, f.y, re);
    re = __fma_rn(c.x, d.x, re);
    re = __fma_rn(-c.y, d.y, re);
    double im = t.x * f.y;
    im = __fma_rn(t.y, f.x, im);
    im = __fma_rn(c.x, d.y, im);
    im = __fma_rn(c.y, d.x, im);
    return make_double2(re, im);
}

// Physical components from split parts (always part q + part q+1).
__device__ __forceinline__ double2 sum_pair(double2 a, double2 b) { return cadd(a, b); }

// Inputs of one H update at cell p (all E sums at level n):
//   ex, ey, ez        E sums at p
//   ex_zm, ey_zm      E_x, E_y at p - e_z   (0 beyond the wall)
//   ex_ym, ez_ym      E_x, E_z at p - e_y
//   ey_xm, ez_xm      E_y, E_z at p - e_x
struct ENbr {
    double2 ex, ey, ez, ex_zm, ey_zm, ex_ym, ez_ym, ey_xm, ez_xm;
};

// Inputs of one E update at cell p (H sums at level n + 1/2):
//   hx, hy, hz        H sums at p
//   hx_zp, hy_zp      H_x, H_y at p + e_z
//   hx_yp, hz_yp      H_x, H_z at p + e_y
//   hy_xp, hz_xp      H_y, H_z at p + e_x
struct HNbr {
    double2 hx, hy, hz, hx_zp, hy_zp, hx_yp, hz_yp, hy_xp, hz_xp;
};

// The six H parts (Eq. 4).  h[]: old parts in / new parts out;
// t[6], c[6]: coefficients of H_xy..H_zy; sxy, syx: Src of H_xy, H_yx.
//   H_xy: +d_z E_y   H_xz: -d_y E_z   H_yx: -d_z E_x
//   H_yz: +d_x E_z   H_zx: +d_y E_x   H_zy: -d_x E_y
__device__ __forceinline__ void update_h(double2 h[6], const double2 t[6],
                                         const double2 c[6], double2 sxy,
                                         double2 syx, const ENbr& e) {
    h[0] = upd_src(h[0], t[0], c[0], csub(e.ey, e.ey_zm), sxy);
    h[1] = upd(h[1], t[1], c[1], csub(e.ez_ym, e.ez));
    h[2] = upd_src(h[2], t[2], c[2], csub(e.ex_zm, e.ex), syx);
    h[3] = upd(h[3], t[3], c[3], csub(e.ez, e.ez_xm));
    h[4] = upd(h[4], t[4], c[4], csub(e.ex, e.ex_ym));
    h[5] = upd(h[5], t[5], c[5], csub(e.ey_xm, e.ey));
}

// The six E parts (Eq. 3 / Eq. 5; the branch lives in the coefficients).
//   E_xy: -d_z H_y   E_xz: +d_y H_z   E_yx: +d_z H_x
//   E_yz: -d_x H_z   E_zx: -d_y H_x   E_zy: +d_x H_y
__device__ __forceinline__ void update_e(double2 e[6], const double2 t[6],
                                         const double2 c[6], double2 sxy,
                                         double2 syx, const HNbr& h) {
    e[0] = upd_src(e[0], t[0], c[0], csub(h.hy, h.hy_zp), sxy);
    e[1] = upd(e[1], t[1], c[1], csub(h.hz_yp, h.hz));
    e[2] = upd_src(e[2], t[2], c[2], csub(h.hx_zp, h.hx), syx);
    e[3] = upd(e[3], t[3], c[3], csub(h.hz, h.hz_xp));
    e[4] = upd(e[4], t[4], c[4], csub(h.hx, h.hx_yp));
    e[5] = upd(e[5], t[5], c[5], csub(h.hy_xp, h.hy));
}

}  // namespace thiim
