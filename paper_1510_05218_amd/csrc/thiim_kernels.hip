// HIP kernels of the THIIM solver for gfx950 (MI355X).
//
// Data layout in HBM: one workspace holding 28 coefficient arrays and two
// 12-array field buffers (A, B), each array [nz][ny][nx] of double2
// (interleaved re/im, x fastest -- the layout of Listings 1 and 2), with a
// common stride S (elements, a multiple of 16 so every array starts on a
// 256-byte boundary).  Lanes run along x, so every array access of a
// wavefront is 64 consecutive 16-byte values (1 KiB, fully coalesced).
//
// Kernels
//   k_coeffs      a0: the 28 coefficient arrays from eps and the PML profiles
//   k_naive_h     a1: H half-step, in place, one HBM sweep (2.5D z streaming)
//   k_naive_e     a2: E half-step, in place, one HBM sweep
//   k_fused       a1+a2 in one HBM pass, A -> B, LDS-staged x-y tile
//   k_resid_*     a5: FP64 residual / norm reduction (deterministic order)
#include "thiim_device.h"
#include "thiim_kernels.h"

namespace thiim {

// ---------------------------------------------------------------------------
// indexing helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long cell(const Geo& g, int k, int j, int i) {
    return ((long long)k * g.ny + j) * g.nx + i;
}

// Maps a global (i, j) that may lie outside [0,nx) x [0,ny) to the cell it
// stands for: wrapped when periodic, false (ghost value 0) when Dirichlet.
__device__ __forceinline__ bool resolve_xy(const Geo& g, int& i, int& j) {
    if (i < 0 || i >= g.nx) {
        if (g.bcx) return false;
        i %= g.nx;
        if (i < 0) i += g.nx;
    }
    if (j < 0 || j >= g.ny) {
        if (g.bcy) return false;
        j %= g.ny;
        if (j < 0) j += g.ny;
    }
    return true;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 d) {
    double den = d.x * d.x + d.y * d.y;
    return make_double2((a.x * d.x + a.y * d.y) / den, (a.y * d.x - a.x * d.y) / den);
}
__device__ __forceinline__ double2 cscale(double s, double2 a) {
    return make_double2(s * a.x, s * a.y);
}

// ---------------------------------------------------------------------------
// a0: coefficients.  Eq. (4) with mu = 1:
//   d_H = e^{iwt/2} + tau sigma*,  t = e^{-iwt/2}/d_H,  c = (tau/h)/d_H,
//   Src = tau S_H / d_H.
// Eq. (3) (eps' > 0):  d = 1 + tau sigma/eps',  t = e^{-iwt}/d,
//   c = tau/(eps' h) e^{-iwt/2}/d,  Src = tau e^{-iwt} S_E / d.
// Eq. (5) (eps' < 0):  d = 1 - tau sigma/eps',  t = e^{iwt}/d,
//   c = -tau/(eps' h) e^{iwt/2}/d,  Src = -tau S_E / d.
// sigma = w eps'' (+ sigma_e(z) on E_xy, E_yx); sigma* = sigma_h(z) on
// H_xy, H_yx and 0 on the other H parts.
// ---------------------------------------------------------------------------
__global__ void k_coeffs(CoefArgs a) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < a.N;
         p += stride) {
        const int k = (int)(p / a.nxy);
        const double2 e = a.eps[p];
        if (!(e.x != 0.0) || !isfinite(e.x) || !isfinite(e.y)) {
            a.flag[0] = 1;
            continue;
        }
        double2* C = a.coef;
        const long long S = a.S;
        // H parts
        const double2 dh0 = a.ph2;  // sigma* = 0
        const double2 dhz = make_double2(a.ph2.x + a.tau * a.sig_h[k], a.ph2.y);
        const double2 th0 = cdiv(a.ph2c, dh0), thz = cdiv(a.ph2c, dhz);
        const double2 ch0 = cdiv(make_double2(a.tau / a.h, 0.0), dh0);
        const double2 chz = cdiv(make_double2(a.tau / a.h, 0.0), dhz);
        for (int q = 0; q < 6; ++q) {
            const bool zax = (q == HXY || q == HYX);
            C[q * S + p] = zax ? thz : th0;
            C[(12 + q) * S + p] = zax ? chz : ch0;
        }
        const double2 sh = cdiv(make_double2(a.tau, 0.0), dhz);
        {
            const double2 s0 = a.src[0] ? a.src[0][p] : czero();
            const double2 s1 = a.src[1] ? a.src[1][p] : czero();
            C[SRC_HXY * S + p] = cmul(sh, s0);
            C[SRC_HYX * S + p] = cmul(sh, s1);
        }
        // E parts
        const double eps = e.x;
        const double sig_mat = a.omega * e.y;
        const double cs = a.tau / (eps * a.h);
        double2 te[2], ce[2], se[2];  // [0]: no PML term, [1]: with sigma_e(z)
        for (int z = 0; z < 2; ++z) {
            const double sg = sig_mat + (z ? a.sig_e[k] : 0.0);
            if (eps > 0.0) {
                const double d = 1.0 + a.tau * sg / eps;
                te[z] = cscale(1.0 / d, a.phc);
                ce[z] = cscale(cs / d, a.ph2c);
                se[z] = cscale(a.tau / d, a.phc);
            } else {
                const double d = 1.0 - a.tau * sg / eps;
                te[z] = cscale(1.0 / d, a.ph);
                ce[z] = cscale(-cs / d, a.ph2);
                se[z] = make_double2(-a.tau / d, 0.0);
            }
        }
        for (int q = 6; q < 12; ++q) {
            const int z = (q == EXY || q == EYX) ? 1 : 0;
            C[q * S + p] = te[z];
            C[(12 + q) * S + p] = ce[z];
        }
        {
            const double2 s2 = a.src[2] ? a.src[2][p] : czero();
            const double2 s3 = a.src[3] ? a.src[3][p] : czero();
            C[SRC_EXY * S + p] = cmul(se[1], s2);
            C[SRC_EYX * S + p] = cmul(se[1], s3);
        }
    }
}

// ---------------------------------------------------------------------------
// helpers loading the six split parts of one cell and forming sums
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load6(const double2* __restrict__ base, long long S,
                                      long long p, double2 v[6]) {
#pragma unroll
    for (int q = 0; q < 6; ++q) v[q] = base[q * S + p];
}
__device__ __forceinline__ void store6(double2* __restrict__ base, long long S,
                                       long long p, const double2 v[6]) {
#pragma unroll
    for (int q = 0; q < 6; ++q) base[q * S + p] = v[q];
}
// coefficients t, c of six parts starting at part q0, and two Src values
__device__ __forceinline__ void load_coef6(const double2* __restrict__ C, long long S,
                                           long long p, int q0, int s0, double2 t[6],
                                           double2 c[6], double2& sa, double2& sb) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        t[q] = C[(q0 + q) * S + p];
        c[q] = C[(12 + q0 + q) * S + p];
    }
    sa = C[s0 * S + p];
    sb = C[(s0 + 1) * S + p];
}

// ---------------------------------------------------------------------------
// a1 naive: H half-step in place.  Thread = (i, j) column, streams z upward
// keeping E_x, E_y of plane k-1 in registers (2.5D streaming).
// Block 64 x 4, grid (nx/64, ny/4, z chunks).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_naive_h(const double2* __restrict__ C,
                                                 double2* __restrict__ F, Geo g,
                                                 int kchunk) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const int k0 = blockIdx.z * kchunk;
    const int k1 = min(g.nz, k0 + kchunk);
    int im = i - 1, jm_i = i, jm = j - 1, im_j = j;
    const bool has_xm = resolve_xy(g, im, im_j);
    const bool has_ym = resolve_xy(g, jm_i, jm);
    const long long S = g.S;
    const double2* E = F + 6 * S;
    double2 ex_zm = czero(), ey_zm = czero();
    if (k0 > 0) {
        const long long q = cell(g, k0 - 1, j, i);
        ex_zm = cadd(E[0 * S + q], E[1 * S + q]);
        ey_zm = cadd(E[2 * S + q], E[3 * S + q]);
    }
    for (int k = k0; k < k1; ++k) {
        const long long p = cell(g, k, j, i);
        double2 ev[6];
        load6(E, S, p, ev);
        ENbr nb;
        nb.ex = cadd(ev[0], ev[1]);
        nb.ey = cadd(ev[2], ev[3]);
        nb.ez = cadd(ev[4], ev[5]);
        nb.ex_zm = ex_zm;
        nb.ey_zm = ey_zm;
        if (has_ym) {
            const long long q = cell(g, k, jm, jm_i);
            nb.ex_ym = cadd(E[0 * S + q], E[1 * S + q]);
            nb.ez_ym = cadd(E[4 * S + q], E[5 * S + q]);
        } else {
            nb.ex_ym = czero();
            nb.ez_ym = czero();
        }
        if (has_xm) {
            const long long q = cell(g, k, im_j, im);
            nb.ey_xm = cadd(E[2 * S + q], E[3 * S + q]);
            nb.ez_xm = cadd(E[4 * S + q], E[5 * S + q]);
        } else {
            nb.ey_xm = czero();
            nb.ez_xm = czero();
        }
        double2 h[6], t[6], c[6], sa, sb;
        load6(F, S, p, h);
        load_coef6(C, S, p, 0, SRC_HXY, t, c, sa, sb);
        update_h(h, t, c, sa, sb, nb);
        store6(F, S, p, h);
        ex_zm = nb.ex;
        ey_zm = nb.ey;
    }
}

// ---------------------------------------------------------------------------
// a2 naive: E half-step in place.  Streams z downward keeping H_x, H_y of
// plane k+1 in registers.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_naive_e(const double2* __restrict__ C,
                                                 double2* __restrict__ F, Geo g,
                                                 int kchunk) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    const int k0 = blockIdx.z * kchunk;
    const int k1 = min(g.nz, k0 + kchunk);
    int ip = i + 1, ip_j = j, jp = j + 1, jp_i = i;
    const bool has_xp = resolve_xy(g, ip, ip_j);
    const bool has_yp = resolve_xy(g, jp_i, jp);
    const long long S = g.S;
    const double2* H = F;
    double2* E = F + 6 * S;
    double2 hx_zp = czero(), hy_zp = czero();
    if (k1 < g.nz) {
        const long long q = cell(g, k1, j, i);
        hx_zp = cadd(H[0 * S + q], H[1 * S + q]);
        hy_zp = cadd(H[2 * S + q], H[3 * S + q]);
    }
    for (int k = k1 - 1; k >= k0; --k) {
        const long long p = cell(g, k, j, i);
        double2 hv[6];
        load6(H, S, p, hv);
        HNbr nb;
        nb.hx = cadd(hv[0], hv[1]);
        nb.hy = cadd(hv[2], hv[3]);
        nb.hz = cadd(hv[4], hv[5]);
        nb.hx_zp = hx_zp;
        nb.hy_zp = hy_zp;
        if (has_yp) {
            const long long q = cell(g, k, jp, jp_i);
            nb.hx_yp = cadd(H[0 * S + q], H[1 * S + q]);
            nb.hz_yp = cadd(H[4 * S + q], H[5 * S + q]);
        } else {
            nb.hx_yp = czero();
            nb.hz_yp = czero();
        }
        if (has_xp) {
            const long long q = cell(g, k, ip_j, ip);
            nb.hy_xp = cadd(H[2 * S + q], H[3 * S + q]);
            nb.hz_xp = cadd(H[4 * S + q], H[5 * S + q]);
        } else {
            nb.hy_xp = czero();
            nb.hz_xp = czero();
        }
        double2 e[6], t[6], c[6], sa, sb;
        load6(E, S, p, e);
        load_coef6(C, S, p, 6, SRC_EXY, t, c, sa, sb);
        update_e(e, t, c, sa, sb, nb);
        store6(E, S, p, e);
        hx_zp = nb.hx;
        hy_zp = nb.hy;
    }
}

// ---------------------------------------------------------------------------
// Fused H+E pass, A -> B (one HBM pass per iteration).
//
// A workgroup owns a TX x TY column tile and streams z.  At step k it
//   1. loads E^n(k) on the tile and its halo ([-1,TX] x [-1,TY]) and puts the
//      component sums E_x, E_y, E_z into LDS;
//   2. computes H^{n+1/2}(k) on the tile and on the +x / +y halo ring
//      ([0,TX] x [0,TY]), stores the tile's parts to B;
//   3. computes E^{n+1}(k-1) on the tile from the H sums of plane k-1 (LDS,
//      written one step earlier) and of plane k (own cell, registers);
//   4. writes the H sums of plane k into LDS for the next step.
// Each thread keeps its own cell for the whole stream (fixed execution to
// data): its old E parts, its z-neighbour sums and its H sums of the previous
// plane stay in registers.  A chunk [k0, k1) of planes recomputes H(k1) (not
// stored) so that chunks are independent.
// ---------------------------------------------------------------------------
template <int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_fused(const double2* __restrict__ C,
                                                  const double2* __restrict__ A,
                                                  double2* __restrict__ B, Geo g,
                                                  int kchunk) {
    constexpr int NT = TX * TY;
    constexpr int EW = TX + 2, EH = TY + 2;  // E region [-1,TX] x [-1,TY]
    constexpr int HW = TX + 1, HH = TY + 1;  // H region [0,TX] x [0,TY]
    constexpr int NE = EW * EH, NH = HW * HH;
    constexpr int NHH = TX + TY + 1;  // H halo cells (column TX, row TY)
    constexpr int NEH = NE - NT;      // E halo cells (H halo first)
    static_assert(NEH <= NT, "halo larger than tile");
    __shared__ double2 Es[3][NE];
    __shared__ double2 Hs[3][NH];

    const long long S = g.S;
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
    const int k0 = blockIdx.z * kchunk;
    const int k1 = min(g.nz, k0 + kchunk);

    // own cell
    const int oi = tid % TX, oj = tid / TX;
    const int eo = (oj + 1) * EW + (oi + 1);
    const int ho = oj * HW + oi;
    int gi = i0 + oi, gj = j0 + oj;
    const bool own_store = gi < g.nx && gj < g.ny;
    const bool own_valid = resolve_xy(g, gi, gj);
    const long long pxy = (long long)gj * g.nx + gi;

    // halo cell (local coordinates), H halo first
    int li = 0, lj = 0;
    if (tid < TY + 1) { li = TX; lj = tid; }
    else if (tid < NHH) { li = tid - (TY + 1); lj = TY; }
    else if (tid < NHH + EW) { li = tid - NHH - 1; lj = -1; }
    else if (tid < NEH) { li = -1; lj = tid - NHH - EW; }
    const bool has_eh = tid < NEH;
    const bool has_hh = tid < NHH;
    const int eh = (lj + 1) * EW + (li + 1);
    const int hh = lj * HW + li;  // valid only if has_hh
    int hgi = i0 + li, hgj = j0 + lj;
    const bool halo_valid = has_eh && resolve_xy(g, hgi, hgj);
    const long long hxy = (long long)hgj * g.nx + hgi;
    const long long plane = (long long)g.nx * g.ny;

    const double2* AE = A + 6 * S;
    double2* BE = B + 6 * S;

    // state carried along z
    double2 eprev[6];  // own E^n parts of plane k-1
    double2 hprev_x = czero(), hprev_y = czero(), hprev_z = czero();
    double2 halo_exm = czero(), halo_eym = czero();
#pragma unroll
    for (int q = 0; q < 6; ++q) eprev[q] = czero();
    if (k0 > 0) {
        if (own_valid) load6(AE, S, (k0 - 1) * plane + pxy, eprev);
        if (has_hh && halo_valid) {
            const long long q = (k0 - 1) * plane + hxy;
            halo_exm = cadd(AE[0 * S + q], AE[1 * S + q]);
            halo_eym = cadd(AE[2 * S + q], AE[3 * S + q]);
        }
    }

    for (int k = k0; k <= k1; ++k) {
        const bool plane_in = k < g.nz;
        double2 ecur[6];
        double2 halo_ex = czero(), halo_ey = czero();
        // ---- phase 1: E^n(k) sums into LDS
        if (plane_in) {
            if (own_valid) {
                load6(AE, S, k * plane + pxy, ecur);
            } else {
#pragma unroll
                for (int q = 0; q < 6; ++q) ecur[q] = czero();
            }
            Es[0][eo] = cadd(ecur[0], ecur[1]);
            Es[1][eo] = cadd(ecur[2], ecur[3]);
            Es[2][eo] = cadd(ecur[4], ecur[5]);
            if (has_eh) {
                double2 ex = czero(), ey = czero(), ez = czero();
                if (halo_valid) {
                    const long long q = k * plane + hxy;
                    ex = cadd(AE[0 * S + q], AE[1 * S + q]);
                    ey = cadd(AE[2 * S + q], AE[3 * S + q]);
                    ez = cadd(AE[4 * S + q], AE[5 * S + q]);
                }
                Es[0][eh] = ex;
                Es[1][eh] = ey;
                Es[2][eh] = ez;
                halo_ex = ex;
                halo_ey = ey;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 6; ++q) ecur[q] = czero();
        }
        __syncthreads();
        // ---- phase 2: H^{n+1/2}(k)
        double2 hx = czero(), hy = czero(), hz = czero();
        double2 hhx = czero(), hhy = czero(), hhz = czero();
        if (plane_in) {
            if (own_valid) {
                ENbr nb;
                nb.ex = Es[0][eo];
                nb.ey = Es[1][eo];
                nb.ez = Es[2][eo];
                nb.ex_zm = cadd(eprev[0], eprev[1]);
                nb.ey_zm = cadd(eprev[2], eprev[3]);
                nb.ex_ym = Es[0][eo - EW];
                nb.ez_ym = Es[2][eo - EW];
                nb.ey_xm = Es[1][eo - 1];
                nb.ez_xm = Es[2][eo - 1];
                const long long p = k * plane + pxy;
                double2 h[6], t[6], c[6], sa, sb;
                load6(A, S, p, h);
                load_coef6(C, S, p, 0, SRC_HXY, t, c, sa, sb);
                update_h(h, t, c, sa, sb, nb);
                if (own_store && k < k1) store6(B, S, p, h);
                hx = cadd(h[0], h[1]);
                hy = cadd(h[2], h[3]);
                hz = cadd(h[4], h[5]);
            }
            if (has_hh && halo_valid) {
                ENbr nb;
                nb.ex = Es[0][eh];
                nb.ey = Es[1][eh];
                nb.ez = Es[2][eh];
                nb.ex_zm = halo_exm;
                nb.ey_zm = halo_eym;
                nb.ex_ym = Es[0][eh - EW];
                nb.ez_ym = Es[2][eh - EW];
                nb.ey_xm = Es[1][eh - 1];
                nb.ez_xm = Es[2][eh - 1];
                const long long p = k * plane + hxy;
                double2 h[6], t[6], c[6], sa, sb;
                load6(A, S, p, h);
                load_coef6(C, S, p, 0, SRC_HXY, t, c, sa, sb);
                update_h(h, t, c, sa, sb, nb);
                hhx = cadd(h[0], h[1]);
                hhy = cadd(h[2], h[3]);
                hhz = cadd(h[4], h[5]);
            }
        }
        // ---- phase 3: E^{n+1}(k-1) on the own cell
        if (k > k0 && own_valid) {
            HNbr nb;
            nb.hx = hprev_x;
            nb.hy = hprev_y;
            nb.hz = hprev_z;
            nb.hx_zp = hx;
            nb.hy_zp = hy;
            nb.hx_yp = Hs[0][ho + HW];
            nb.hz_yp = Hs[2][ho + HW];
            nb.hy_xp = Hs[1][ho + 1];
            nb.hz_xp = Hs[2][ho + 1];
            const long long p = (k - 1) * plane + pxy;
            double2 t[6], c[6], sa, sb;
            load_coef6(C, S, p, 6, SRC_EXY, t, c, sa, sb);
            update_e(eprev, t, c, sa, sb, nb);
            if (own_store) store6(BE, S, p, eprev);
        }
        __syncthreads();
        // ---- phase 4: H sums of plane k into LDS, shift the z state
        Hs[0][ho] = hx;
        Hs[1][ho] = hy;
        Hs[2][ho] = hz;
        if (has_hh) {
            Hs[0][hh] = hhx;
            Hs[1][hh] = hhy;
            Hs[2][hh] = hhz;
        }
        hprev_x = hx;
        hprev_y = hy;
        hprev_z = hz;
        halo_exm = halo_ex;
        halo_eym = halo_ey;
#pragma unroll
        for (int q = 0; q < 6; ++q) eprev[q] = ecur[q];
    }
}

// ---------------------------------------------------------------------------
// a5: residual.  Per cell: |P(B - A)|^2 and |P B|^2 summed over the six
// physical components (P: sum of each split pair).  Block partial sums, then
// one block reduces the partials in a fixed order: deterministic FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double* sh) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_resid_partial(const double2* __restrict__ A,
                                                       const double2* __restrict__ B,
                                                       long long S, long long N,
                                                       double* __restrict__ part) {
    __shared__ double sh[256];
    double r2 = 0.0, b2 = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < N;
         p += stride) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const double2 a0 = A[(2 * c) * S + p], a1 = A[(2 * c + 1) * S + p];
            const double2 b0 = B[(2 * c) * S + p], b1 = B[(2 * c + 1) * S + p];
            const double2 d = cadd(csub(b0, a0), csub(b1, a1));
            const double2 pb = cadd(b0, b1);
            r2 = __fma_rn(d.x, d.x, r2);
            r2 = __fma_rn(d.y, d.y, r2);
            b2 = __fma_rn(pb.x, pb.x, b2);
            b2 = __fma_rn(pb.y, pb.y, b2);
        }
    }
    const double s1 = block_sum(r2, sh);
    const double s2 = block_sum(b2, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1;
        part[2 * blockIdx.x + 1] = s2;
    }
}

__global__ __launch_bounds__(256) void k_resid_final(const double* __restrict__ part,
                                                     int nblk, double* __restrict__ out) {
    __shared__ double sh[256];
    double r2 = 0.0, b2 = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        r2 += part[2 * b];
        b2 += part[2 * b + 1];
    }
    const double s1 = block_sum(r2, sh);
    const double s2 = block_sum(b2, sh);
    if (threadIdx.x == 0) {
        out[0] = s1;
        out[1] = s2;
    }
}

// Fill / copy helpers (kernels rather than memset so callers may capture them
// in graphs).
__global__ void k_fill_zero(double2* __restrict__ p, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = czero();
}

__global__ void k_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                       long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int grid_1d(long long n, int block) {
    long long b = (n + block - 1) / block;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_coeffs(const CoefArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_coeffs, dim3(grid_1d(a.N, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

static int nchunks(const Geo& g, int kchunk) { return (g.nz + kchunk - 1) / kchunk; }

hipError_t launch_naive(const double2* C, double2* F, const Geo& g, int kchunk,
                        hipStream_t s) {
    dim3 grid((g.nx + 63) / 64, (g.ny + 3) / 4, nchunks(g, kchunk));
    hipLaunchKernelGGL(k_naive_h, grid, dim3(64, 4), 0, s, C, F, g, kchunk);
    hipLaunchKernelGGL(k_naive_e, grid, dim3(64, 4), 0, s, C, F, g, kchunk);
    return hipGetLastError();
}

hipError_t launch_fused(const double2* C, const double2* A, double2* B, const Geo& g,
                        int tile_x, int tile_y, int kchunk, hipStream_t s) {
    dim3 grid((g.nx + tile_x - 1) / tile_x, (g.ny + tile_y - 1) / tile_y, nchunks(g, kchunk));
    if (tile_x == 64 && tile_y == 8)
        hipLaunchKernelGGL((k_fused<64, 8>), grid, dim3(512), 0, s, C, A, B, g, kchunk);
    else if (tile_x == 32 && tile_y == 8)
        hipLaunchKernelGGL((k_fused<32, 8>), grid, dim3(256), 0, s, C, A, B, g, kchunk);
    else if (tile_x == 64 && tile_y == 4)
        hipLaunchKernelGGL((k_fused<64, 4>), grid, dim3(256), 0, s, C, A, B, g, kchunk);
    else if (tile_x == 16 && tile_y == 16)
        hipLaunchKernelGGL((k_fused<16, 16>), grid, dim3(256), 0, s, C, A, B, g, kchunk);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_resid(const double2* A, const double2* B, long long S, long long N,
                        double* part, int nblk, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_resid_partial, dim3(nblk), dim3(256), 0, s, A, B, S, N, part);
    hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(256), 0, s, part, nblk, out);
    return hipGetLastError();
}

hipError_t launch_fill_zero(double2* p, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_1d(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_copy(const double2* src, double2* dst, long long n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(grid_1d(n, 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace thiim
