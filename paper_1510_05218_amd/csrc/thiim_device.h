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
__device__ __forceinline__ float2 cadd(float2 a, float2 b) {
    return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) {
    return make_float2(a.x - b.x, a.y - b.y);
}
template <class V> __device__ __forceinline__ V vzero();
template <> __device__ __forceinline__ double2 vzero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ float2 vzero<float2>() { return make_float2(0.0f, 0.0f); }

// t * f + src + c * d  (complex), fixed operation order
__device__ __forceinline__ double2 upd_src(double2 f, double2 t, double2 c, double2 d,
                                           double2 src) {
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
__device__ __forceinline__ double2 upd(double2 f, double2 t, double2 c, double2 d) {
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

// complex64 forms (inner sweeps of the mixed-precision solver)
__device__ __forceinline__ float2 upd_src(float2 f, float2 t, float2 c, float2 d, float2 src) {
    float re = __fmaf_rn(t.x, f.x, src.x);
    re = __fmaf_rn(-t.y, f.y, re);
    re = __fmaf_rn(c.x, d.x, re);
    re = __fmaf_rn(-c.y, d.y, re);
    float im = __fmaf_rn(t.x, f.y, src.y);
    im = __fmaf_rn(t.y, f.x, im);
    im = __fmaf_rn(c.x, d.y, im);
    im = __fmaf_rn(c.y, d.x, im);
    return make_float2(re, im);
}
__device__ __forceinline__ float2 upd(float2 f, float2 t, float2 c, float2 d) {
    float re = t.x * f.x;
    re = __fmaf_rn(-t.y, f.y, re);
    re = __fmaf_rn(c.x, d.x, re);
    re = __fmaf_rn(-c.y, d.y, re);
    float im = t.x * f.y;
    im = __fmaf_rn(t.y, f.x, im);
    im = __fmaf_rn(c.x, d.y, im);
    im = __fmaf_rn(c.y, d.x, im);
    return make_float2(re, im);
}

// Inputs of one H update at cell p (all E sums at level n):
//   ex, ey, ez        E sums at p
//   ex_zm, ey_zm      E_x, E_y at p - e_z   (0 beyond the wall)
//   ex_ym, ez_ym      E_x, E_z at p - e_y
//   ey_xm, ez_xm      E_y, E_z at p - e_x
template <class V>
struct ENbrT {
    V ex, ey, ez, ex_zm, ey_zm, ex_ym, ez_ym, ey_xm, ez_xm;
};
using ENbr = ENbrT<double2>;

// Inputs of one E update at cell p (H sums at level n + 1/2):
//   hx, hy, hz        H sums at p
//   hx_zp, hy_zp      H_x, H_y at p + e_z
//   hx_yp, hz_yp      H_x, H_z at p + e_y
//   hy_xp, hz_xp      H_y, H_z at p + e_x
template <class V>
struct HNbrT {
    V hx, hy, hz, hx_zp, hy_zp, hx_yp, hz_yp, hy_xp, hz_xp;
};
using HNbr = HNbrT<double2>;

// The six H parts (Eq. 4).  h[]: old parts in / new parts out;
// t[6], c[6]: coefficients of H_xy..H_zy; src[q] enters part q when bit q of
// MASK is set (the paper's layout: MASK = 0b000101, Src of H_xy and H_yx).
//   H_xy: +d_z E_y   H_xz: -d_y E_z   H_yx: -d_z E_x
//   H_yz: +d_x E_z   H_zx: +d_y E_x   H_zy: -d_x E_y
template <int MASK, class V>
__device__ __forceinline__ void update_h_t(V h[6], const V t[6], const V c[6], const V src[6],
                                           const ENbrT<V>& e) {
    const V d[6] = {csub(e.ey, e.ey_zm), csub(e.ez_ym, e.ez), csub(e.ex_zm, e.ex),
                    csub(e.ez, e.ez_xm), csub(e.ex, e.ex_ym), csub(e.ey_xm, e.ey)};
#pragma unroll
    for (int q = 0; q < 6; ++q)
        h[q] = ((MASK >> q) & 1) ? upd_src(h[q], t[q], c[q], d[q], src[q])
                                 : upd(h[q], t[q], c[q], d[q]);
}

// The six E parts (Eq. 3 / Eq. 5; the branch lives in the coefficients).
//   E_xy: -d_z H_y   E_xz: +d_y H_z   E_yx: +d_z H_x
//   E_yz: -d_x H_z   E_zx: -d_y H_x   E_zy: +d_x H_y
// The signed differences s_q (G(p + e) - G(p)) of the six E parts.
template <class V>
__device__ __forceinline__ void e_diffs(const HNbrT<V>& h, V d[6]) {
    d[0] = csub(h.hy, h.hy_zp);
    d[1] = csub(h.hz_yp, h.hz);
    d[2] = csub(h.hx_zp, h.hx);
    d[3] = csub(h.hz, h.hz_xp);
    d[4] = csub(h.hx, h.hx_yp);
    d[5] = csub(h.hy_xp, h.hy);
}

template <int MASK, class V>
__device__ __forceinline__ void update_e_t(V e[6], const V t[6], const V c[6], const V src[6],
                                           const HNbrT<V>& h) {
    V d[6];
    e_diffs(h, d);
#pragma unroll
    for (int q = 0; q < 6; ++q)
        e[q] = ((MASK >> q) & 1) ? upd_src(e[q], t[q], c[q], d[q], src[q])
                                 : upd(e[q], t[q], c[q], d[q]);
}

constexpr int SRC_MASK_Z = 0b000101;  // Src on the two z-difference parts
constexpr int SRC_MASK_ALL = 0b111111;

// FP64 forms with the two Src values of the paper's layout.
__device__ __forceinline__ void update_h(double2 h[6], const double2 t[6], const double2 c[6],
                                         double2 sxy, double2 syx, const ENbr& e) {
    const double2 src[6] = {sxy, czero(), syx, czero(), czero(), czero()};
    update_h_t<SRC_MASK_Z>(h, t, c, src, e);
}
__device__ __forceinline__ void update_e(double2 e[6], const double2 t[6], const double2 c[6],
                                         double2 sxy, double2 syx, const HNbr& h) {
    const double2 src[6] = {sxy, czero(), syx, czero(), czero(), czero()};
    update_e_t<SRC_MASK_Z>(e, t, c, src, h);
}

}  // namespace thiim
