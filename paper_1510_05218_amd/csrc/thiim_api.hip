// C-ABI of the THIIM library: context, validation, workspace layout and the
// dispatch of one iteration to the naive, fused or temporally blocked sweeps.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/thiim.h"
#include "thiim_kernels.h"

using thiim::Geo;

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int hip_fail(hipError_t e, const char* where) {
    return fail(THIIM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr int kResidBlocks = 1024;
constexpr size_t kHeaderBytes = 4096;  // flag, reduction output

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Cells added to every array stride (17 x 256 bytes of complex128).  On a
// power-of-two grid the arrays would otherwise all start at the same offset
// modulo the HBM channel interleave, so the 25-52 streams of one sweep hit
// the same channels together; an odd multiple of 256 bytes spreads them
// (7-8% faster sweeps at 512^3).
constexpr long long kStridePad = 272;

// Workgroups of one residual-forming fused pass, bounded so that their
// partial sums fit the workspace: the largest column-tile count of the fused
// tiles, times 16 z chunks (at least kResidBlocks, the plain reduction's grid).
int resid_blocks(const thiim_grid* g) {
    const int tiles[4][2] = {{64, 8}, {32, 8}, {64, 4}, {16, 16}};
    long long m = 0;
    for (auto& t : tiles)
        m = std::max(m, (long long)((g->nx + t[0] - 1) / t[0]) * ((g->ny + t[1] - 1) / t[1]));
    return (int)std::max<long long>(kResidBlocks, 16 * m);
}

struct Layout {
    long long N, S;   // cells, array stride (double2)
    int resid_max;    // workgroups of a residual pass (resid_blocks)
    size_t off_sig;   // 2*nz doubles
    size_t off_part;  // 2*resid_max doubles
    size_t off_plane; // nz PlaneCoef
    size_t off_coef;  // full: 28 arrays; compact: eps + 4 Src arrays
    size_t off_a, off_b;
    size_t off_r32, off_d32;  // mixed precision: 12 + 24 complex64 arrays
    size_t off_acc32;         // mixed precision: 12 complex64 arrays (window sum)
    size_t off_rt32;          // mixed precision: 12 complex64 arrays (r_T)
    size_t off_ce, off_p32;   // mixed precision: per-cell float4 records, nz plane rows
    size_t off_lam, off_g;    // adjoint: 4 x 12 + 3 complex128 arrays
    size_t total;
};

Layout layout_of(const thiim_grid* g) {
    Layout L;
    L.N = (long long)g->nx * g->ny * g->nz;
    L.S = (long long)align_up((size_t)L.N, kAlign / 16) + kStridePad;
    size_t off = kHeaderBytes;
    L.off_sig = off;
    off = align_up(off + 2 * sizeof(double) * g->nz, kAlign);
    L.resid_max = resid_blocks(g);
    L.off_part = off;
    off = align_up(off + 2 * sizeof(double) * L.resid_max, kAlign);
    L.off_plane = off;
    off = align_up(off + sizeof(thiim::PlaneCoef) * g->nz, kAlign);
    L.off_coef = off;
    off += (size_t)(g->storage == THIIM_STORAGE_COMPACT ? 5 : 28) * L.S * 16;
    L.off_a = off;
    off += (size_t)12 * L.S * 16;
    L.off_b = off;
    off += (size_t)12 * L.S * 16;
    L.off_r32 = L.off_d32 = L.off_acc32 = L.off_rt32 = L.off_ce = L.off_p32 = 0;
    if (g->precision == THIIM_PRECISION_MIXED) {
        L.off_r32 = off;
        off += (size_t)12 * L.S * 8;
        L.off_d32 = off;
        off += (size_t)24 * L.S * 8;
        L.off_acc32 = off;
        off += (size_t)12 * L.S * 8;
        L.off_rt32 = off;
        off += (size_t)12 * L.S * 8;
        L.off_ce = off;
        off += (size_t)L.S * 16;
        L.off_p32 = off;
        off = align_up(off + sizeof(thiim::PlaneCoef32) * g->nz, kAlign);
    }
    L.off_lam = L.off_g = 0;
    if (g->adjoint) {
        L.off_lam = off;
        off += (size_t)48 * L.S * 16;
        L.off_g = off;
        off += (size_t)3 * L.S * 16;
    }
    L.total = off;
    return L;
}

int check_grid(const thiim_grid* g) {
    if (!g) return fail(THIIM_EINVAL, "grid is NULL");
    if (g->nx < 2 || g->ny < 2 || g->nz < 2)
        return fail(THIIM_EINVAL, "nx, ny, nz must each be >= 2");
    if ((long long)g->nx * g->ny * g->nz > (1LL << 40))
        return fail(THIIM_EINVAL, "grid too large");
    if ((g->bc_x != THIIM_PERIODIC && g->bc_x != THIIM_DIRICHLET) ||
        (g->bc_y != THIIM_PERIODIC && g->bc_y != THIIM_DIRICHLET))
        return fail(THIIM_EINVAL, "bc_x / bc_y must be PERIODIC or DIRICHLET");
    if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(THIIM_EINVAL, "h must be > 0");
    if (!(g->tau > 0.0) || !(g->tau <= g->h / std::sqrt(3.0) * (1.0 + 1e-12)))
        return fail(THIIM_EINVAL, "tau must satisfy 0 < tau <= h/sqrt(3) (CFL)");
    if (g->kernel < THIIM_KERNEL_AUTO || g->kernel > THIIM_KERNEL_BLOCKED)
        return fail(THIIM_EINVAL, "unknown kernel");
    if (g->precision != THIIM_PRECISION_FP64 && g->precision != THIIM_PRECISION_MIXED)
        return fail(THIIM_EINVAL, "precision must be FP64 or MIXED");
    if (g->precision == THIIM_PRECISION_MIXED && g->storage != THIIM_STORAGE_COMPACT)
        return fail(THIIM_EINVAL, "mixed precision needs the compact coefficient storage");
    if (g->t_block < 0 || g->t_block > (g->precision == THIIM_PRECISION_MIXED ? 3 : 2))
        return fail(THIIM_EINVAL, "t_block must be 0 (auto), 1 or 2 (3 with mixed precision)");
    if (g->storage != THIIM_STORAGE_FULL && g->storage != THIIM_STORAGE_COMPACT)
        return fail(THIIM_EINVAL, "storage must be FULL or COMPACT");
    if ((long long)g->nx * g->ny * 16 > 0xFFFFFFFFLL)
        return fail(THIIM_EINVAL, "an x-y plane must hold fewer than 2^28 cells");
    if (g->z_chunk < 0) return fail(THIIM_EINVAL, "z_chunk must be >= 0");
    if (g->adjoint != 0 && g->adjoint != 1) return fail(THIIM_EINVAL, "adjoint must be 0 or 1");
    if (g->adjoint && g->storage != THIIM_STORAGE_COMPACT)
        return fail(THIIM_EINVAL, "the adjoint gradient needs the compact coefficient storage");
    const bool tile_auto = g->tile_x == 0 && g->tile_y == 0;
    if (g->kernel == THIIM_KERNEL_BLOCKED) {
        if (!tile_auto && !(g->tile_x == 64 && (g->tile_y == 8 || g->tile_y == 6)) &&
            !(g->tile_x == 32 && g->tile_y == 16))
            return fail(THIIM_EINVAL, "blocked kernel: tile must be 0x0 (auto), 64x8, 64x6 or "
                                      "32x16 (region columns x rows)");
    } else {
        const bool tile_ok = (g->tile_x == 64 && g->tile_y == 8) ||
                             (g->tile_x == 32 && g->tile_y == 8) ||
                             (g->tile_x == 64 && g->tile_y == 4) ||
                             (g->tile_x == 16 && g->tile_y == 16);
        if (!tile_auto && !tile_ok)
            return fail(THIIM_EINVAL, "tile must be 0x0 (auto), 64x8, 32x8, 64x4 or 16x16");
    }
    return THIIM_OK;
}

}  // namespace

struct thiim_ctx {
    thiim_grid g;
    Geo geo;
    Layout L;
    thiim::CoefView cv;
    double omega;
    hipStream_t stream;
    int device;
    char* ws;
    double2* coef;
    double2* F[2];
    int cur;  // index of the buffer holding the current state
    double* sig_dev;
    double* part;
    double* out;  // [2] reduction output
    int* flag;
    double phi0_norm;
    long long iters;
    int kernel;  // resolved THIIM_KERNEL_*
    int tile_x, tile_y, z_chunk;      // fused sweep
    int t_block, region_x, region_y, bz_chunk;  // blocked sweep
    float2* r32;                                // mixed precision buffers
    float2* d32[2];
    float2* acc32;                // window sum of the inner passes
    float2* rt32;                 // r_T = (I + M) r, the two-sweep passes' source
    float4* ce32;                 // per-cell complex64 E-coefficient records
    thiim::PlaneCoef32* p32;      // per-plane complex64 H coefficients
    int inner_t, inner_rx, inner_ry, inner_chunk;
    int ncu;          // compute units of the device
    double2* lam[4];  // adjoint buffers
    double2* gadj;    // adjoint source, 3 arrays
};

namespace {

// Compute units of the current device (256 on an MI355X).
int cu_count() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n < 1)
        n = 256;
    return n;
}

// z planes per workgroup stream.  The sweeps keep one workgroup resident per
// CU (their LDS and registers allow no second), so a launch of W workgroups
// runs in ceil(W / CUs) rounds, each about as long as one chunk plus ~3
// planes of pipeline fill; choose the chunk count (chunks of >= 16 planes)
// that minimises rounds x (chunk + 3).  At 512^3 the blocked sweep has 817
// tiles and this picks 5 chunks of 103 planes; chunks of 86 to 171 planes
// measure within a few per cent of each other there.
int auto_chunk(const thiim_grid& g, long long tiles, int ncu) {
    int best = 1;
    double best_cost = INFINITY;
    const int max_nch = g.nz / 16 > 1 ? g.nz / 16 : 1;
    for (int nch = 1; nch <= max_nch; ++nch) {
        const int zc = (g.nz + nch - 1) / nch;
        const long long rounds = (tiles * nch + ncu - 1) / ncu;
        const double cost = (double)rounds * (zc + 3);
        if (cost < best_cost * (1.0 - 1e-9)) {
            best_cost = cost;
            best = nch;
        }
    }
    return (g.nz + best - 1) / best;
}

int resolve_tiles(thiim_ctx* c) {
    const thiim_grid& g = c->g;
    // auto: the two-iteration blocked sweep when the coefficients are compact
    // (its second stage then re-reads 16 B per cell), the fused sweep for the
    // 28-array layout (where the second stage would re-read 448 B per cell)
    if (g.kernel == THIIM_KERNEL_AUTO)
        c->kernel = g.storage == THIIM_STORAGE_COMPACT ? THIIM_KERNEL_BLOCKED : THIIM_KERNEL_FUSED;
    else
        c->kernel = g.kernel;
    if (c->kernel != THIIM_KERNEL_BLOCKED && g.tile_x != 0) {
        c->tile_x = g.tile_x;
        c->tile_y = g.tile_y;
    } else if (g.nx >= 48) {
        c->tile_x = 64;
        c->tile_y = 8;
    } else if (g.nx >= 24) {
        c->tile_x = 32;
        c->tile_y = 8;
    } else {
        c->tile_x = 16;
        c->tile_y = 16;
    }
    const long long tiles = (long long)((g.nx + c->tile_x - 1) / c->tile_x) *
                            ((g.ny + c->tile_y - 1) / c->tile_y);
    c->z_chunk = g.z_chunk > 0 ? g.z_chunk : auto_chunk(g, tiles, c->ncu);
    c->t_block = g.t_block > 0 ? (g.t_block > 2 ? 2 : g.t_block) : 2;
    const bool btile = c->kernel == THIIM_KERNEL_BLOCKED && g.tile_x != 0;
    const bool compact = g.storage == THIIM_STORAGE_COMPACT;
    c->region_x = btile ? g.tile_x : (compact ? 32 : 64);
    c->region_y = btile ? g.tile_y : (compact ? 16 : 8);
    const int ox = c->region_x - 2 * c->t_block, oy = c->region_y - 2 * c->t_block;
    const long long btiles = (long long)((g.nx + ox - 1) / ox) * ((g.ny + oy - 1) / oy);
    c->bz_chunk = g.z_chunk > 0 ? g.z_chunk : auto_chunk(g, btiles, c->ncu);
    // complex64 inner sweeps of the mixed solver: two per pass on 32 x 32
    // regions (four waves per SIMD), or three per pass on 32 x 16 regions
    // when t_block = 3 is asked for (two waves per SIMD; 12% slower per sweep
    // at 512^3)
    c->inner_t = g.t_block == 3 ? 3 : 2;
    c->inner_rx = 32;
    c->inner_ry = c->inner_t == 2 ? 32 : 16;
    const int iox = c->inner_rx - 2 * c->inner_t, ioy = c->inner_ry - 2 * c->inner_t;
    const long long itiles = (long long)((g.nx + iox - 1) / iox) * ((g.ny + ioy - 1) / ioy);
    c->inner_chunk = g.z_chunk > 0 ? g.z_chunk : auto_chunk(g, itiles, c->ncu);
    return THIIM_OK;
}

// One THIIM iteration from buffer `src` into buffer `dst` (src != dst).
hipError_t one_pass(thiim_ctx* c, int src, int dst) {
    return thiim::launch_fused(c->cv, c->F[src], c->F[dst], c->geo, c->tile_x, c->tile_y,
                               c->z_chunk, c->stream);
}

int reduce_pair(thiim_ctx* c, const double2* A, const double2* B, int c0, double* r2,
                double* b2);

// Phi(F[src]) into F[dst] by the fused pass, with the residual sums of the
// iteration (||P(F[dst] - F[src])||^2, ||P F[dst]||^2) left in c->out.
hipError_t residual_pass(thiim_ctx* c, int src, int dst, hipStream_t s) {
    return thiim::launch_fused_res(c->cv, c->F[src], c->F[dst], c->geo, c->tile_x, c->tile_y,
                                   c->z_chunk, c->part, c->L.resid_max, c->out, s);
}

// c->out to the host (synchronising)
int read_out(thiim_ctx* c, double* r2, double* b2) {
    double host[2];
    hipError_t e = hipMemcpyAsync(host, c->out, sizeof(host), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "residual copy");
    *r2 = host[0];
    *b2 = host[1];
    return THIIM_OK;
}

// r2 = ||P(B - A)||^2, b2 = ||P B||^2 over physical components c0..5
// (synchronising)
int reduce_pair(thiim_ctx* c, const double2* A, const double2* B, int c0, double* r2,
                double* b2) {
    hipError_t e = thiim::launch_resid(A, B, c->L.S, c->L.N, c0, c->part, kResidBlocks, c->out,
                                       c->stream);
    if (e != hipSuccess) return hip_fail(e, "residual launch");
    double host[2];
    e = hipMemcpyAsync(host, c->out, sizeof(host), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(e, "residual copy");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "residual sync");
    *r2 = host[0];
    *b2 = host[1];
    return THIIM_OK;
}

}  // namespace

extern "C" {

int thiim_workspace_bytes(const thiim_grid* g, size_t* bytes) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!bytes) return fail(THIIM_EINVAL, "bytes is NULL");
    *bytes = layout_of(g).total;
    return THIIM_OK;
}

int thiim_create(const thiim_grid* g, const thiim_coeffs* m, double omega, void* workspace,
                 size_t workspace_bytes, thiim_ctx** out) {
    if (!out) return fail(THIIM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_grid(g);
    if (rc) return rc;
    if (!m || !m->eps || !m->sigma_e || !m->sigma_h)
        return fail(THIIM_EINVAL, "coeffs, eps, sigma_e and sigma_h are required");
    if (!(omega > 0.0) || !std::isfinite(omega)) return fail(THIIM_EINVAL, "omega must be > 0");
    for (int k = 0; k < g->nz; ++k) {
        if (!std::isfinite(m->sigma_e[k]) || !std::isfinite(m->sigma_h[k]) ||
            m->sigma_e[k] < 0.0 || m->sigma_h[k] < 0.0)
            return fail(THIIM_EINVAL, "PML conductivities must be finite and >= 0");
    }
    const Layout L = layout_of(g);
    if (!workspace) return fail(THIIM_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % kAlign) return fail(THIIM_EINVAL, "workspace must be 256-byte aligned");
    if (workspace_bytes < L.total)
        return fail(THIIM_ENOMEM, "workspace smaller than thiim_workspace_bytes()");
    if (((uintptr_t)m->eps) % 16) return fail(THIIM_EINVAL, "eps must be 16-byte aligned");
    for (int s = 0; s < 4; ++s)
        if (m->src[s] && ((uintptr_t)m->src[s]) % 16)
            return fail(THIIM_EINVAL, "source arrays must be 16-byte aligned");

    thiim_ctx* c = new (std::nothrow) thiim_ctx();
    if (!c) return fail(THIIM_EINVAL, "out of host memory");
    c->g = *g;
    c->L = L;
    c->omega = omega;
    c->stream = (hipStream_t)g->stream;
    (void)hipGetDevice(&c->device);
    c->ncu = cu_count();
    c->ws = (char*)workspace;
    c->flag = (int*)c->ws;
    c->out = (double*)(c->ws + 256);
    c->sig_dev = (double*)(c->ws + L.off_sig);
    c->part = (double*)(c->ws + L.off_part);
    c->coef = (double2*)(c->ws + L.off_coef);
    c->F[0] = (double2*)(c->ws + L.off_a);
    c->F[1] = (double2*)(c->ws + L.off_b);
    c->r32 = L.off_r32 ? (float2*)(c->ws + L.off_r32) : nullptr;
    c->d32[0] = L.off_d32 ? (float2*)(c->ws + L.off_d32) : nullptr;
    c->d32[1] = L.off_d32 ? c->d32[0] + 12 * L.S : nullptr;
    c->acc32 = L.off_acc32 ? (float2*)(c->ws + L.off_acc32) : nullptr;
    c->rt32 = L.off_rt32 ? (float2*)(c->ws + L.off_rt32) : nullptr;
    c->ce32 = L.off_ce ? (float4*)(c->ws + L.off_ce) : nullptr;
    c->p32 = L.off_p32 ? (thiim::PlaneCoef32*)(c->ws + L.off_p32) : nullptr;
    c->lam[0] = L.off_lam ? (double2*)(c->ws + L.off_lam) : nullptr;
    for (int i = 1; i < 4; ++i) c->lam[i] = L.off_lam ? c->lam[0] + 12 * i * L.S : nullptr;
    c->gadj = L.off_g ? (double2*)(c->ws + L.off_g) : nullptr;
    c->cur = 0;
    c->iters = 0;
    c->geo = Geo{g->nx, g->ny, g->nz, g->bc_x, g->bc_y, L.S};
    resolve_tiles(c);

    auto bail = [&](int status) {
        delete c;
        return status;
    };
    hipError_t e;
    e = hipMemsetAsync(c->ws, 0, kHeaderBytes, c->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "memset"));
    e = hipMemcpyAsync(c->sig_dev, m->sigma_e, sizeof(double) * g->nz, hipMemcpyHostToDevice,
                       c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->sig_dev + g->nz, m->sigma_h, sizeof(double) * g->nz,
                           hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "profile copy"));

    const bool compact = g->storage == THIIM_STORAGE_COMPACT;
    thiim::CoefConst K;
    K.tau = g->tau;
    K.h = g->h;
    K.omega = omega;
    const double wt = omega * g->tau;
    K.ph = make_double2(std::cos(wt), std::sin(wt));
    K.phc = make_double2(std::cos(wt), -std::sin(wt));
    K.ph2 = make_double2(std::cos(wt / 2), std::sin(wt / 2));
    K.ph2c = make_double2(std::cos(wt / 2), -std::sin(wt / 2));
    thiim::PlaneCoef* P = (thiim::PlaneCoef*)(c->ws + L.off_plane);
    double2* cbase = (double2*)(c->ws + L.off_coef);
    c->cv.compact = compact ? 1 : 0;
    c->cv.C = compact ? nullptr : cbase;
    c->cv.eps = compact ? cbase : nullptr;
    c->cv.src = compact ? cbase + L.S : cbase + 24 * L.S;
    c->cv.P = P;
    c->cv.S = L.S;
    c->cv.K = K;
    c->coef = cbase;

    thiim::BuildArgs a;
    a.eps_in = (const double2*)m->eps;
    a.sig_e = c->sig_dev;
    a.sig_h = c->sig_dev + g->nz;
    for (int s = 0; s < 4; ++s) a.src_in[s] = (const double2*)m->src[s];
    a.C = compact ? nullptr : cbase;
    a.eps_out = compact ? cbase : nullptr;
    a.src_out = (double2*)c->cv.src;
    a.P = P;
    a.S = L.S;
    a.N = L.N;
    a.nxy = (long long)g->nx * g->ny;
    a.nz = g->nz;
    a.K = K;
    a.flag = c->flag;
    e = thiim::launch_build(a, compact, c->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "coefficient launch"));
    // x = 0; the other buffer needs no clearing: every pass writes all of its
    // output's cells before anything reads them
    e = thiim::launch_fill_zero(c->F[0], 12 * L.S, c->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "zero fields"));
    int flag = 0;
    std::vector<thiim::PlaneCoef> planes(g->nz);
    e = hipMemcpyAsync(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(planes.data(), P, sizeof(thiim::PlaneCoef) * g->nz,
                           hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "create sync"));
    if (flag) return bail(fail(THIIM_EINVAL, "eps has a non-finite value or eps' == 0"));

    if (c->ce32) {
        e = thiim::launch_prep32(c->cv, c->geo, c->ce32, c->p32, c->stream);
        if (e != hipSuccess) return bail(hip_fail(e, "complex64 coefficient launch"));
    }

    // ||P Phi(0)||, one iteration from the zero state.  Phi(0) is zero except
    // on the planes that carry a source (H = Src_H, E) and the plane below
    // each (E reads H one plane up), so the residual pass runs on that range
    // of planes only, as a grid of its own: the zero planes around it are
    // what its z walls assume.
    int smin = g->nz, smax = -1;
    for (int k = 0; k < g->nz; ++k)
        if (planes[k].has_src) {
            smin = std::min(smin, k);
            smax = std::max(smax, k);
        }
    double r2 = 0, b2 = 0;
    if (smax >= 0) {
        const int k0 = std::max(0, smin - 1), k1 = smax + 1;
        const long long off = (long long)k0 * g->nx * g->ny;
        thiim::CoefView v = c->cv;
        if (v.C) v.C += off;
        if (v.eps) v.eps += off;
        v.src += off;
        v.P += k0;
        thiim::Geo gr = c->geo;
        gr.nz = k1 - k0;
        e = thiim::launch_fused_res(v, c->F[0] + off, c->F[1] + off, gr, c->tile_x, c->tile_y,
                                    c->z_chunk, c->part, c->L.resid_max, c->out, c->stream);
        if (e != hipSuccess) return bail(hip_fail(e, "phi(0) launch"));
        rc = read_out(c, &r2, &b2);
        if (rc) return bail(rc);
    }
    c->phi0_norm = std::sqrt(b2);
    if (!std::isfinite(c->phi0_norm)) return bail(fail(THIIM_EINVAL, "non-finite source response"));
    *out = c;
    return THIIM_OK;
}

int thiim_iterate(thiim_ctx* c, int n) {
    if (!c) return fail(THIIM_EINVAL, "ctx is NULL");
    if (n < 0) return fail(THIIM_EINVAL, "n must be >= 0");
    for (int it = 0; it < n; ++it) {
        hipError_t e;
        if (c->kernel == THIIM_KERNEL_NAIVE) {
            e = thiim::launch_naive(c->cv, c->F[c->cur], c->geo, c->z_chunk, c->stream);
        } else if (c->kernel == THIIM_KERNEL_BLOCKED && c->t_block > 1 &&
                   n - it >= c->t_block) {
            e = thiim::launch_blocked(c->cv, c->F[c->cur], c->F[1 - c->cur], c->geo,
                                      c->t_block, c->region_x, c->region_y, c->bz_chunk,
                                      c->stream);
            c->cur = 1 - c->cur;
            it += c->t_block - 1;
            c->iters += c->t_block - 1;
        } else {
            e = one_pass(c, c->cur, 1 - c->cur);
            c->cur = 1 - c->cur;
        }
        if (e != hipSuccess) return hip_fail(e, "iterate launch");
        c->iters++;
    }
    return THIIM_OK;
}

int thiim_residual(thiim_ctx* c, double* rel_res) {
    if (!c || !rel_res) return fail(THIIM_EINVAL, "ctx / rel_res is NULL");
    const int other = 1 - c->cur;
    hipError_t e = residual_pass(c, c->cur, other, c->stream);
    if (e != hipSuccess) return hip_fail(e, "residual pass");
    double r2 = 0, b2 = 0;
    int rc = read_out(c, &r2, &b2);
    if (rc) return rc;
    const double r = std::sqrt(r2) / (c->phi0_norm > 0 ? c->phi0_norm : 1.0);
    *rel_res = r;
    if (!std::isfinite(r)) return fail(THIIM_EDIVERGED, "residual is not finite");
    return THIIM_OK;
}

namespace {

// Mixed-precision defect correction (see THIIM_PRECISION_MIXED).
//
// Each step: FP64 sweep Phi(x), r = Phi(x) - x (FP64 norms; complex64 copy
// with the invisible split differences dropped), d = r then d <- M d + r in
// complex64, x += d in FP64.
//
// Rounding a correction to complex64 also puts single-precision noise into
// the modes that one iteration only rotates by l = e^{-iw tau} (curl-free H
// where sigma* = 0, curl-free E in lossless cells).  For such a mode the
// inner sum d = sum_k M^k r oscillates instead of converging to
// r / (1 - l), so a correction only rotates it: left alone, the noise of all
// corrections piles up there and holds the residual near 1e-6 |x| / |Phi(0)|.
// The correction therefore averages d over the last Kp passes, one rotation
// period 2 pi / (w tau) of those modes: the average of l^k over a period is
// ~0, so the averaged d carries r / (1 - l) for them (to a factor 1/(2 Kp))
// while every other mode mu keeps |weight| <= 1 (the average of mu^k), i.e.
// nothing is amplified.  The inner passes of the window sum their d into a
// complex64 buffer as they store it, and x += sum / Kp follows in FP64 once
// per correction.
//
// check_every > 0 fixes the inner sweeps per correction; 0 adapts it: start
// at max(64, 2 Kp T) and double (up to kMaxInner) while a correction gains
// less than kWeak.
constexpr double kWeak = 0.3;
constexpr int kMaxInner = 1 << 15;
// A solve is declared divergent when its residual exceeds kGrowth times the
// smallest residual it has reached (a convergent THIIM iteration can grow
// transiently, by far less; a medium with gain, eps'' < 0, grows without
// bound).
constexpr double kGrowth = 1e6;

// One inner pass of the context from A into B: with two sweeps per pass the
// source is r_T (rt32) at the last stage, with three r (r32) at every stage.
hipError_t launch_pass32(thiim_ctx* c, const float2* A, float2* B, int acc_mode, hipStream_t s) {
    const bool last = c->inner_t == 2;
    return thiim::launch_inner32(c->cv, c->ce32, c->p32, last ? c->rt32 : c->r32, last, A, B,
                                 c->acc32, acc_mode, c->geo, c->inner_t, c->inner_rx,
                                 c->inner_ry, c->inner_chunk, s);
}

// r_T = (I + M) r for the two-sweep passes: one pass with source r at both
// stages from d = 0 (d32[1] cleared first).  Nothing for three-sweep passes.
hipError_t launch_rt(thiim_ctx* c, hipStream_t s) {
    if (c->inner_t != 2) return hipSuccess;
    hipError_t e = thiim::launch_fill_zero((double2*)c->d32[1], 6 * c->L.S, s);
    if (e != hipSuccess) return e;
    return thiim::launch_inner32(c->cv, c->ce32, c->p32, c->r32, false, c->d32[1], c->rt32,
                                 nullptr, 0, c->geo, 2, c->inner_rx, c->inner_ry,
                                 c->inner_chunk, s);
}

int solve_mixed(thiim_ctx* c, double tol, int max_it, int inner, int* iters, double* rel_res) {
    const int other = 1 - c->cur;
    const int T = c->inner_t;
    const double wt = c->omega * c->g.tau;
    int Kp = (int)std::lround(2.0 * M_PI / (wt * T));
    if (Kp < 1) Kp = 1;
    const bool adaptive = inner <= 0;
    int m = adaptive ? (2 * Kp * T > 64 ? 2 * Kp * T : 64) : inner;
    int done = 0;
    double r = INFINITY, prev = INFINITY, best = INFINITY;
    for (;;) {
        // FP64: Phi(x) into the other buffer, r = Phi(x) - x (complex64 copy)
        hipError_t e = one_pass(c, c->cur, other);
        if (e != hipSuccess) return hip_fail(e, "mixed: residual sweep");
        e = thiim::launch_defect(c->F[c->cur], c->F[other], c->r32, c->cv.P, c->L.S, c->L.N,
                                 (long long)c->g.nx * c->g.ny, c->part, kResidBlocks, c->out,
                                 c->stream);
        if (e != hipSuccess) return hip_fail(e, "mixed: defect");
        double host[2];
        e = hipMemcpyAsync(host, c->out, sizeof(host), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(e, "mixed: residual sync");
        done += 1;
        r = std::sqrt(host[0]) / (c->phi0_norm > 0 ? c->phi0_norm : 1.0);
        if (!std::isfinite(r) || r > kGrowth * best) {
            if (iters) *iters = done;
            if (rel_res) *rel_res = r;
            return fail(THIIM_EDIVERGED, std::isfinite(r) ? "residual grew 1e6-fold: diverging"
                                                          : "residual is not finite");
        }
        best = std::min(best, r);
        if (r <= tol || done >= max_it) break;
        if (adaptive && std::isfinite(prev) && r > kWeak * prev && m < kMaxInner) m *= 2;
        // complex64: d = r, then passes of d <- M d + r; the last Kp averaged
        int passes = (m - 1 + T - 1) / T;
        if (passes < Kp) passes = Kp;
        e = launch_rt(c, c->stream);
        if (e == hipSuccess) e = thiim::launch_copy32(c->r32, c->d32[0], c->L.S, c->L.N, c->stream);
        int di = 0;
        for (int p = 0; e == hipSuccess && p < passes; ++p) {
            // the last Kp passes also sum what they store into acc32
            const int acc_mode = p < passes - Kp ? 0 : (p == passes - Kp ? 1 : 2);
            e = launch_pass32(c, c->d32[di], c->d32[1 - di], acc_mode, c->stream);
            di = 1 - di;
        }
        // x += (window sum) / Kp in FP64
        if (e == hipSuccess)
            e = thiim::launch_accum(c->F[c->cur], c->acc32, 1.0 / Kp, c->cv.P, 0.5,
                                    (long long)c->g.nx * c->g.ny, c->L.S, c->L.N, c->stream);
        if (e != hipSuccess) return hip_fail(e, "mixed: inner sweeps");
        done += passes * T;           // sweeps run (d = r is a copy)
        c->iters += 1 + passes * T;   // equivalent plain iterations
        prev = r;
    }
    if (iters) *iters = done;
    if (rel_res) *rel_res = r;
    if (r > tol) return fail(THIIM_ENOTCONV, "iteration limit reached before tolerance");
    return THIIM_OK;
}

}  // namespace

int thiim_solve(thiim_ctx* c, double tol, int max_it, int check_every, int* iters,
                double* rel_res) {
    if (!c) return fail(THIIM_EINVAL, "ctx is NULL");
    if (c->g.precision == THIIM_PRECISION_MIXED) {
        if (!(tol > 0.0) || max_it < 0 || check_every < 0)
            return fail(THIIM_EINVAL, "need tol > 0, max_it >= 0, check_every >= 0");
        return solve_mixed(c, tol, max_it, check_every, iters, rel_res);
    }
    if (!(tol > 0.0) || max_it < 0 || check_every < 1)
        return fail(THIIM_EINVAL, "need tol > 0, max_it >= 0, check_every >= 1");
    int done = 0;
    double r = INFINITY;
    int rc = thiim_residual(c, &r);
    double best = r;
    while (rc == THIIM_OK && r > tol && done < max_it) {
        const int step = check_every < max_it - done ? check_every : max_it - done;
        rc = thiim_iterate(c, step);
        if (rc) break;
        done += step;
        rc = thiim_residual(c, &r);
        if (rc == THIIM_OK && r > kGrowth * best)
            rc = fail(THIIM_EDIVERGED, "residual grew 1e6-fold: diverging");
        best = std::min(best, r);
    }
    if (iters) *iters = done;
    if (rel_res) *rel_res = r;
    if (rc) return rc;
    if (r > tol) return fail(THIIM_ENOTCONV, "iteration limit reached before tolerance");
    return THIIM_OK;
}

int thiim_adjoint_grad(thiim_ctx* c, const double* weight, double tol, int max_it,
                       int check_every, double* grad_eps, double* J, int* iters,
                       double* rel_res) {
    if (!c) return fail(THIIM_EINVAL, "ctx is NULL");
    if (!c->lam[0]) return fail(THIIM_EINVAL, "the context was created without adjoint = 1");
    if (!weight || !grad_eps) return fail(THIIM_EINVAL, "weight / grad_eps is NULL");
    if (((uintptr_t)weight) % 8 || ((uintptr_t)grad_eps) % 16)
        return fail(THIIM_EINVAL, "weight must be 8-byte and grad_eps 16-byte aligned");
    if (max_it < 0 || (tol > 0.0 && check_every < 1) || !std::isfinite(tol))
        return fail(THIIM_EINVAL, "need max_it >= 0, finite tol and check_every >= 1");
    const int other = 1 - c->cur;
    const long long S = c->L.S, N = c->L.N;
    // Phi(x): its H parts are the H half-step of x
    hipError_t e = one_pass(c, c->cur, other);
    if (e != hipSuccess) return hip_fail(e, "adjoint: forward sweep");
    e = thiim::launch_adj_source(c->F[c->cur], c->cv.eps, weight, S, N, c->gadj, c->part,
                                 kResidBlocks, c->out, c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint: source");
    double host[2];
    e = hipMemcpyAsync(host, c->out, sizeof(host), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint: objective sync");
    const double jval = host[0];
    e = thiim::launch_fill_zero(c->lam[0], 24 * S, c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint: zero");
    int li = 0, done = 0, rc = THIIM_OK;
    double r = 0.0, norm0 = 0.0;
    auto sweep = [&](int src, int dst, const double2* G, bool dense) {
        return thiim::launch_adjoint(c->cv, c->lam[src], c->lam[dst], G, dense, c->geo,
                                     c->tile_x, c->tile_y, c->z_chunk, c->stream);
    };
    // ||P(lam_b - lam_a)_E|| / ||P g_E|| (P: split-pair sum, R19)
    auto measure = [&](int a, int b, double* rr) {
        double r2 = 0, b2 = 0;
        int rc2 = reduce_pair(c, c->lam[a], c->lam[b], 3, &r2, &b2);
        if (rc2) return rc2;
        if (norm0 == 0.0) norm0 = std::sqrt(b2);  // first call: lam_a = 0, lam_b = g
        *rr = norm0 > 0 ? std::sqrt(r2) / norm0 : 0.0;
        return THIIM_OK;
    };
    if (!(tol > 0.0)) {
        // exactly max_it transposed iterations from lam = 0
        for (int it = 0; it < max_it; ++it) {
            e = sweep(li, 1 - li, c->gadj, false);
            if (e != hipSuccess) return hip_fail(e, "adjoint: sweep");
            li = 1 - li;
            ++done;
            if (it == 0) {
                rc = measure(1 - li, li, &r);
                if (rc) return rc;
            }
        }
        if (max_it > 1) {
            rc = measure(1 - li, li, &r);
            if (rc) return rc;
        }
    } else {
        // Defect correction with period-averaged corrections (as in the
        // mixed-precision solver, in FP64): r = M^T lam + g - lam, then
        // d <- M^T d + r and lam += the mean of d over the last Kp sweeps, one
        // rotation period of the modes an iteration rotates by e^{-iw tau}.
        // Compared with the plain transposed iteration this removes their
        // rotating part and damps the slowly decaying modes of the first PML
        // planes, where sigma is small.  Buffers: lam = 0, Phi = 1, d = 2, 3.
        int Kp = (int)std::lround(2.0 * M_PI / (c->omega * c->g.tau));
        if (Kp < 1) Kp = 1;
        int m = check_every > 2 * Kp ? check_every : 2 * Kp;
        double prev = INFINITY, best = INFINITY;
        for (;;) {
            e = sweep(0, 1, c->gadj, false);
            if (e != hipSuccess) return hip_fail(e, "adjoint: sweep");
            ++done;
            rc = measure(0, 1, &r);
            if (rc) return rc;
            if (!std::isfinite(r) || r > kGrowth * best) {
                if (iters) *iters = done;
                if (rel_res) *rel_res = r;
                return fail(THIIM_EDIVERGED, std::isfinite(r)
                                                 ? "adjoint residual grew 1e6-fold: diverging"
                                                 : "adjoint residual is not finite");
            }
            best = std::min(best, r);
            if (r <= tol || done >= max_it) break;
            if (std::isfinite(prev) && r > 0.3 * prev && m < (1 << 15)) m *= 2;
            prev = r;
            e = thiim::launch_sub(c->lam[0], c->lam[1], S, N, c->stream);  // r
            if (c->ce32) {
                // mixed-precision context: complex64 inner sweeps (its r32 and
                // d32 buffers), two per pass of the temporally blocked
                // transposed sweep, averaged over the passes of one rotation
                // period; the defect and lam in FP64
                if (e == hipSuccess) e = thiim::launch_to32(c->lam[1], c->r32, S, N, c->stream);
                constexpr int T2 = 2;
                // the passes add G_T = (I + M^T) r at their last stage: one pass
                // with source r at both stages from d = 0 (into rt32, free while
                // the adjoint runs)
                if (e == hipSuccess)
                    e = thiim::launch_fill_zero((double2*)c->d32[1], 6 * S, c->stream);
                if (e == hipSuccess)
                    e = thiim::launch_adjoint32_blocked(c->cv, c->ce32, c->p32, c->d32[1],
                                                        c->rt32, c->r32, false, nullptr, 0,
                                                        c->geo, T2, 32, 16, c->bz_chunk,
                                                        c->stream);
                if (e == hipSuccess) e = thiim::launch_copy32(c->r32, c->d32[0], S, N, c->stream);
                // the passes' z chunk, for their 32 x 24 regions
                constexpr int aox = 32 - 2 * T2, aoy = 24 - 2 * T2;
                const long long atiles =
                    (long long)((c->g.nx + aox - 1) / aox) * ((c->g.ny + aoy - 1) / aoy);
                const int achunk =
                    c->g.z_chunk > 0 ? c->g.z_chunk : auto_chunk(c->g, atiles, c->ncu);
                int Kq = (int)std::lround(2.0 * M_PI / (c->omega * c->g.tau * T2));
                if (Kq < 1) Kq = 1;
                const int passes = (m + T2 - 1) / T2 > Kq ? (m + T2 - 1) / T2 : Kq;
                // the last Kq passes sum their output into acc32 as they go; one
                // FP64 kernel then adds the mean to lam
                int di = 0;
                for (int p = 0; e == hipSuccess && p < passes; ++p) {
                    const int left = passes - p;
                    const int acc_mode = left > Kq ? 0 : (left == Kq ? 1 : 2);
                    e = thiim::launch_adjoint32_blocked(c->cv, c->ce32, c->p32, c->d32[di],
                                                        c->d32[1 - di], c->rt32, true, c->acc32,
                                                        acc_mode, c->geo, T2, 32, 24, achunk,
                                                        c->stream);
                    di = 1 - di;
                }
                if (e == hipSuccess)
                    e = thiim::launch_accum(c->lam[0], c->acc32, 1.0 / Kq, c->cv.P, 1.0,
                                            (long long)c->g.nx * c->g.ny, S, N,
                                            c->stream);
                done += passes * T2 - m;  // counted below as m
            } else {
                if (e == hipSuccess)
                    e = thiim::launch_copy(c->lam[1], c->lam[2], 12 * S, c->stream);
                int di = 2;
                for (int p = 0; e == hipSuccess && p < m; ++p) {
                    e = sweep(di, 5 - di, c->lam[1], true);
                    di = 5 - di;
                    if (e == hipSuccess && p >= m - Kp)
                        e = thiim::launch_axpy(c->lam[0], c->lam[di], 1.0 / Kp, S, N, c->stream);
                }
            }
            if (e != hipSuccess) return hip_fail(e, "adjoint: correction");
            done += m;
        }
        li = 0;
    }
    e = thiim::launch_adj_grad(c->cv, c->F[c->cur], c->F[other], c->lam[li], weight, c->geo,
                               (double2*)grad_eps, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint: gradient");
    if (J) *J = jval;
    if (iters) *iters = done;
    if (rel_res) *rel_res = r;
    if (tol > 0.0 && r > tol)
        return fail(THIIM_ENOTCONV, "adjoint: iteration limit reached before tolerance");
    return THIIM_OK;
}

int thiim_get_fields(thiim_ctx* c, double* dst) {
    if (!c || !dst) return fail(THIIM_EINVAL, "ctx / dst is NULL");
    for (int q = 0; q < 12; ++q) {
        hipError_t e = hipMemcpyAsync(dst + 2 * q * c->L.N, c->F[c->cur] + q * c->L.S,
                                      16 * c->L.N, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(e, "get_fields");
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? THIIM_OK : hip_fail(e, "get_fields sync");
}

int thiim_set_fields(thiim_ctx* c, const double* src) {
    if (!c || !src) return fail(THIIM_EINVAL, "ctx / src is NULL");
    for (int q = 0; q < 12; ++q) {
        hipError_t e = hipMemcpyAsync(c->F[c->cur] + q * c->L.S, src + 2 * q * c->L.N,
                                      16 * c->L.N, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(e, "set_fields");
    }
    c->iters = 0;
    return THIIM_OK;
}

int thiim_get_coeffs(thiim_ctx* c, double* dst) {
    if (!c || !dst) return fail(THIIM_EINVAL, "ctx / dst is NULL");
    hipError_t e = hipSuccess;
    if (c->cv.compact) {
        e = thiim::launch_expand(c->cv, c->geo, (double2*)dst, c->stream);
        if (e != hipSuccess) return hip_fail(e, "get_coeffs expand");
    } else {
        for (int q = 0; q < 28; ++q) {
            e = hipMemcpyAsync(dst + 2 * q * c->L.N, c->coef + q * c->L.S, 16 * c->L.N,
                               hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return hip_fail(e, "get_coeffs");
        }
    }
    e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? THIIM_OK : hip_fail(e, "get_coeffs sync");
}

// ---------------------------------------------------------------------------
// Auto-tuner: a capacity / traffic model prunes the sweep configurations,
// the survivors are timed on the live context.
// ---------------------------------------------------------------------------
namespace {

struct Candidate {
    int kernel, tx, ty, chunk;
    double model_ms;
};

// Modelled time of one iteration: HBM bytes per cell (tile halos and z-chunk
// overlap included) at 5 TB/s, stretched by the launch's round quantisation:
// with one resident workgroup per CU, W workgroups of kchunk planes occupy
// ceil(W / CUs) rounds of (kchunk + 3) plane-steps on every CU.
double model_ms(const thiim_grid& g, const Candidate& c, int ncu) {
    const double N = (double)g.nx * g.ny * g.nz;
    const bool compact = g.storage == THIIM_STORAGE_COMPACT;
    const double reads = compact ? 13.0 : 36.0;  // arrays read per cell and pass
    double bytes, wgs;
    if (c.kernel == THIIM_KERNEL_BLOCKED) {
        const int T = 2, ox = c.tx - 2 * T, oy = c.ty - 2 * T;
        const double halo = (double)c.tx * c.ty / ((double)ox * oy);
        const double zover = 1.0 + (double)(T - 1) / c.chunk;
        // full storage: every stage re-reads its 28 coefficient arrays
        const double coef_extra = compact ? 0.0 : 28.0 * (T - 1);
        bytes = 16.0 * ((reads * zover + coef_extra) * halo + 12.0) / T;
        wgs = (double)((g.nx + ox - 1) / ox) * ((g.ny + oy - 1) / oy) *
              ((g.nz + c.chunk - 1) / c.chunk);
    } else {
        const double nt = (double)c.tx * c.ty;
        const double halo = 6.0 * (2.0 * c.tx + 2.0 * c.ty + 4.0) / nt;  // E parts of the ring
        bytes = 16.0 * (reads + halo + 12.0 + 12.0 / c.chunk);
        wgs = (double)((g.nx + c.tx - 1) / c.tx) * ((g.ny + c.ty - 1) / c.ty) *
              ((g.nz + c.chunk - 1) / c.chunk);
    }
    const double rounds = std::ceil(wgs / ncu);
    const double quant = rounds * ncu * (c.chunk + 3.0) / (wgs * c.chunk);
    return bytes * N / 5.0e12 * quant * 1e3;
}

void apply(thiim_ctx* c, const Candidate& k) {
    if (k.kernel == THIIM_KERNEL_BLOCKED) {
        c->kernel = THIIM_KERNEL_BLOCKED;
        c->t_block = 2;
        c->region_x = k.tx;
        c->region_y = k.ty;
        c->bz_chunk = k.chunk;
    } else {
        c->kernel = THIIM_KERNEL_FUSED;
        c->tile_x = k.tx;
        c->tile_y = k.ty;
        c->z_chunk = k.chunk;
    }
}

// One pass of the configuration from the current state into the other
// buffer (the state does not advance).
hipError_t trial_pass(thiim_ctx* c, const Candidate& k) {
    const int src = c->cur, dst = 1 - c->cur;
    if (k.kernel == THIIM_KERNEL_BLOCKED)
        return thiim::launch_blocked(c->cv, c->F[src], c->F[dst], c->geo, 2, k.tx, k.ty, k.chunk,
                                     c->stream);
    return thiim::launch_fused(c->cv, c->F[src], c->F[dst], c->geo, k.tx, k.ty, k.chunk,
                               c->stream);
}

}  // namespace

int thiim_autotune(thiim_ctx* c, int trial_iters, thiim_tuning* out) {
    if (!c) return fail(THIIM_EINVAL, "ctx is NULL");
    if (trial_iters < 1) return fail(THIIM_EINVAL, "trial_iters must be >= 1");
    const thiim_grid& g = c->g;
    std::vector<Candidate> all;
    std::vector<int> chunks = {16, 32, 64, 128, 256, g.nz};
    // the round-quantisation choice for each sweep geometry, and its neighbours
    for (long long tl : {(long long)((g.nx + 27) / 28) * ((g.ny + 11) / 12),
                         (long long)((g.nx + 59) / 60) * ((g.ny + 3) / 4),
                         (long long)((g.nx + 63) / 64) * ((g.ny + 7) / 8)}) {
        const int zc = auto_chunk(g, tl, c->ncu);
        const int nch = (g.nz + zc - 1) / zc;
        for (int d = -1; d <= 1; ++d)
            if (nch + d >= 1) chunks.push_back((g.nz + nch + d - 1) / (nch + d));
    }
    chunks.push_back(c->z_chunk);
    chunks.push_back(c->bz_chunk);
    std::sort(chunks.begin(), chunks.end());
    chunks.erase(std::unique(chunks.begin(), chunks.end()), chunks.end());
    const int regions[3][2] = {{32, 16}, {64, 8}, {64, 6}};
    const int tiles[4][2] = {{64, 8}, {32, 8}, {64, 4}, {16, 16}};
    for (int zc : chunks) {
        // chunks of at least 4 planes; a grid of 2 or 3 planes is one chunk
        if (zc > g.nz || (zc < 4 && zc != g.nz)) continue;
        for (auto& r : regions) all.push_back({THIIM_KERNEL_BLOCKED, r[0], r[1], zc, 0.0});
        for (auto& t : tiles) all.push_back({THIIM_KERNEL_FUSED, t[0], t[1], zc, 0.0});
    }
    if (all.empty()) return fail(THIIM_EINVAL, "autotune: no sweep configuration fits the grid");
    for (auto& k : all) k.model_ms = model_ms(g, k, c->ncu);
    std::sort(all.begin(), all.end(),
              [](const Candidate& a, const Candidate& b) { return a.model_ms < b.model_ms; });
    const double cut = 1.3 * all.front().model_ms;
    std::vector<Candidate> keep;
    for (auto& k : all)
        if (k.model_ms <= cut && keep.size() < 10) keep.push_back(k);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(THIIM_EDEVICE, "autotune: event create");
    int best = -1;
    double best_ms = INFINITY;
    int rc = THIIM_OK;
    for (size_t i = 0; i < keep.size() && rc == THIIM_OK; ++i) {
        const Candidate& k = keep[i];
        const int per = k.kernel == THIIM_KERNEL_BLOCKED ? 2 : 1;
        const int passes = (trial_iters + per - 1) / per;
        hipError_t e = trial_pass(c, k);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int p = 0; e == hipSuccess && p < passes; ++p) e = trial_pass(c, k);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune trial");
            break;
        }
        const double per_it = ms / (passes * per);
        if (per_it < best_ms) {
            best_ms = per_it;
            best = (int)i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (best < 0) return fail(THIIM_EDEVICE, "autotune: no trial produced a timing");
    apply(c, keep[best]);
    if (out) {
        out->kernel = keep[best].kernel;
        out->tile_x = keep[best].tx;
        out->tile_y = keep[best].ty;
        out->t_block = keep[best].kernel == THIIM_KERNEL_BLOCKED ? 2 : 1;
        out->z_chunk = keep[best].chunk;
        out->ms_per_iteration = best_ms;
        out->model_ms = keep[best].model_ms;
        out->candidates = (int)all.size();
        out->timed = (int)keep.size();
        out->one_for_all_ms = best_ms;
        out->per_grid_ms = 0.0;
        out->per_grid = 0;
    }
    return THIIM_OK;
}

int thiim_apply_tuning(thiim_ctx* c, const thiim_tuning* t) {
    if (!c || !t) return fail(THIIM_EINVAL, "ctx / tuning is NULL");
    const bool blocked = t->kernel == THIIM_KERNEL_BLOCKED;
    if (!blocked && t->kernel != THIIM_KERNEL_FUSED)
        return fail(THIIM_EINVAL, "apply_tuning: kernel must be FUSED or BLOCKED");
    const bool ok = blocked ? ((t->tile_x == 32 && t->tile_y == 16) ||
                               (t->tile_x == 64 && (t->tile_y == 8 || t->tile_y == 6)))
                            : ((t->tile_x == 64 && (t->tile_y == 8 || t->tile_y == 4)) ||
                               (t->tile_x == 32 && t->tile_y == 8) ||
                               (t->tile_x == 16 && t->tile_y == 16));
    if (!ok) return fail(THIIM_EINVAL, "apply_tuning: tile / region not supported");
    if (t->z_chunk < 1 || t->z_chunk > c->g.nz)
        return fail(THIIM_EINVAL, "apply_tuning: z_chunk must be in [1, nz]");
    apply(c, Candidate{t->kernel, t->tile_x, t->tile_y, t->z_chunk, 0.0});
    return THIIM_OK;
}

// ---------------------------------------------------------------------------
// Batches: many contexts (uneven grids, compact storage, one stream) advanced
// together, one batched launch per sweep configuration and pass, the passes
// of a fixed number of iterations captured once in a HIP graph and replayed.
// ---------------------------------------------------------------------------
}  // extern "C"

struct thiim_batch {
    struct Group {
        int blocked;         // 1: blocked T = 2 passes, 0: fused passes
        int tx, ty;          // region / tile
        std::vector<int> members;
        int total;           // tiles of all members
        thiim::BatchItem* dev[2];  // item arrays by parity
        int par;
    };
    std::vector<thiim_ctx*> ctx;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    unsigned int* queue;  // device work queue of the persistent batched passes
    int ncu;
    std::vector<char> active;
    std::vector<Group> groups;
    bool dirty;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int graph_iters;
    std::vector<int> graph_par;
    int static_dev;  // device whose static scratch this batch holds, or -1
};

namespace {

constexpr int kGraphIters = 64;  // iterations per captured graph (a multiple of 4)

constexpr size_t batch_items_bytes(int n) {
    return align_up((size_t)2 * n * sizeof(thiim::BatchItem), kAlign);
}
constexpr size_t batch_items32_bytes(int n) {
    return align_up((size_t)2 * n * sizeof(thiim::BatchItem32), kAlign);
}
// item arrays (both kinds), then the 9 counters of the device work queue
constexpr size_t batch_bytes(int n) {
    return batch_items_bytes(n) + batch_items32_bytes(n) + kAlign;
}
unsigned int* batch_queue(thiim_batch* b, int n) {
    return (unsigned int*)(b->ws + batch_items_bytes(n) + batch_items32_bytes(n));
}

void drop_graph(thiim_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

thiim::BatchItem item_of(thiim_ctx* c, int parity, int blocked, int tx, int ty, int* tiles) {
    thiim::BatchItem it;
    it.cv = c->cv;
    const int src = parity ? 1 - c->cur : c->cur;
    it.A = c->F[src];
    it.B = c->F[1 - src];
    it.g = c->geo;
    const int ox = blocked ? tx - 4 : tx, oy = blocked ? ty - 4 : ty;
    it.kchunk = blocked ? c->bz_chunk : c->z_chunk;
    it.ntx = (c->g.nx + ox - 1) / ox;
    it.nty = (c->g.ny + oy - 1) / oy;
    it.ntz = (c->g.nz + it.kchunk - 1) / it.kchunk;
    it.tile_begin = 0;
    *tiles = it.ntx * it.nty * it.ntz;
    return it;
}

// Groups the active problems by sweep configuration and uploads the item
// arrays of both parities (synchronising).
int rebuild(thiim_batch* b) {
    drop_graph(b);
    b->groups.clear();
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        if (!b->active[i]) continue;
        thiim_ctx* c = b->ctx[i];
        const int blocked = c->kernel == THIIM_KERNEL_BLOCKED && c->t_block == 2;
        const int tx = blocked ? c->region_x : c->tile_x, ty = blocked ? c->region_y : c->tile_y;
        auto it = std::find_if(b->groups.begin(), b->groups.end(), [&](const thiim_batch::Group& gr) {
            return gr.blocked == blocked && gr.tx == tx && gr.ty == ty;
        });
        if (it == b->groups.end()) {
            b->groups.push_back(thiim_batch::Group{blocked, tx, ty, {}, 0, {nullptr, nullptr}, 0});
            it = b->groups.end() - 1;
        }
        it->members.push_back((int)i);
    }
    thiim::BatchItem* base = (thiim::BatchItem*)b->ws;
    std::vector<thiim::BatchItem> host;
    for (auto& gr : b->groups) {
        gr.par = 0;
        for (int par = 0; par < 2; ++par) {
            gr.dev[par] = base + host.size();
            int t = 0;
            for (int m : gr.members) {
                int tiles = 0;
                thiim::BatchItem it = item_of(b->ctx[m], par, gr.blocked, gr.tx, gr.ty, &tiles);
                it.tile_begin = t;
                t += tiles;
                host.push_back(it);
            }
            gr.total = t;
        }
    }
    if (!host.empty()) {
        hipError_t e = hipMemcpyAsync(b->ws, host.data(), host.size() * sizeof(thiim::BatchItem),
                                      hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch: item upload");
    }
    b->dirty = false;
    return THIIM_OK;
}

// Enqueues `iters` iterations of every active problem (iters even for the
// blocked groups to stay in step; an odd remainder runs one fused pass per
// blocked member).  Updates parities and context states.
hipError_t enqueue(thiim_batch* b, int iters) {
    hipError_t e = hipSuccess;
    for (auto& gr : b->groups) {
        const int passes = gr.blocked ? iters / 2 : iters;
        for (int p = 0; e == hipSuccess && p < passes; ++p) {
            e = gr.blocked ? thiim::launch_blocked_batch(gr.dev[gr.par], (int)gr.members.size(),
                                                         gr.total, 2, gr.tx, gr.ty, b->queue,
                                                         b->ncu, b->stream)
                           : thiim::launch_fused_batch(gr.dev[gr.par], (int)gr.members.size(),
                                                       gr.total, gr.tx, gr.ty, b->queue, b->ncu,
                                                       b->stream);
            gr.par ^= 1;
            for (int m : gr.members) b->ctx[m]->cur ^= 1;
        }
        if (gr.blocked && (iters & 1)) {
            for (int m : gr.members) {
                thiim_ctx* c = b->ctx[m];
                if (e == hipSuccess) e = one_pass(c, c->cur, 1 - c->cur);
                c->cur ^= 1;
            }
            gr.par ^= 1;
        }
    }
    return e;
}

int batch_iterate(thiim_batch* b, int n) {
    if (b->dirty) {
        int rc = rebuild(b);
        if (rc) return rc;
    }
    int left = n;
    // the null stream cannot be captured: eager launches there
    while (b->stream && left >= kGraphIters) {
        std::vector<int> par;
        for (auto& gr : b->groups) par.push_back(gr.par);
        if (!b->exec || par != b->graph_par) {
            drop_graph(b);
            hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "batch: begin capture");
            hipError_t el = enqueue(b, kGraphIters);
            e = hipStreamEndCapture(b->stream, &b->graph);
            if (el != hipSuccess) return hip_fail(el, "batch: captured launch");
            if (e != hipSuccess) return hip_fail(e, "batch: end capture");
            e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return hip_fail(e, "batch: instantiate");
            b->graph_par = par;  // kGraphIters even: parities return to `par`
            // the capture recorded the passes without running them; the state
            // flips it applied are undone by the even pass counts
        }
        hipError_t e = hipGraphLaunch(b->exec, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch: graph launch");
        left -= kGraphIters;
    }
    if (left > 0) {
        hipError_t e = enqueue(b, left);
        if (e != hipSuccess) return hip_fail(e, "batch: launch");
    }
    for (size_t i = 0; i < b->ctx.size(); ++i)
        if (b->active[i]) b->ctx[i]->iters += n;
    return THIIM_OK;
}

// Residual of every active problem (one fused pass and reduction each, one
// synchronisation).
int batch_residual(thiim_batch* b, std::vector<double>& r) {
    const size_t n = b->ctx.size();
    std::vector<double> host(2 * n, 0.0);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < n && e == hipSuccess; ++i) {
        if (!b->active[i]) continue;
        thiim_ctx* c = b->ctx[i];
        e = residual_pass(c, c->cur, 1 - c->cur, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&host[2 * i], c->out, 2 * sizeof(double), hipMemcpyDeviceToHost,
                               b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch: residual");
    r.assign(n, NAN);
    for (size_t i = 0; i < n; ++i) {
        if (!b->active[i]) continue;
        const double p0 = b->ctx[i]->phi0_norm;
        r[i] = std::sqrt(host[2 * i]) / (p0 > 0 ? p0 : 1.0);
    }
    return THIIM_OK;
}

// Mixed-precision batch solve: the defect-correction steps of solve_mixed
// for all active problems at once -- per problem the FP64 residual sweep and
// defect, then the complex64 inner passes of all problems with the same T as
// one batched launch per pass (the inner phase of a step captured once in a
// HIP graph per active set), each problem averaging its own last Kp passes
// into x.  All problems run the same number of inner sweeps per step: m, or
// with m = 0 the adaptive count of solve_mixed driven by the slowest problem.
int batch_solve_mixed(thiim_batch* b, double tol, int max_it, int m_user,
                      std::vector<int>& done, std::vector<double>& r, bool& diverged) {
    const size_t n = b->ctx.size();
    std::vector<int> Kp(n), T(n);
    int m = 64;
    for (size_t i = 0; i < n; ++i) {
        thiim_ctx* c = b->ctx[i];
        T[i] = c->inner_t;
        Kp[i] = (int)std::lround(2.0 * M_PI / (c->omega * c->g.tau * T[i]));
        if (Kp[i] < 1) Kp[i] = 1;
        if (2 * Kp[i] * T[i] > m) m = 2 * Kp[i] * T[i];
    }
    if (m_user > 0) m = m_user;
    std::vector<double> prev(n, INFINITY), best(n, INFINITY);
    thiim::BatchItem32* base = (thiim::BatchItem32*)(b->ws + batch_items_bytes((int)n));
    struct G32 {
        int T;
        std::vector<int> members;
        int total;
        thiim::BatchItem32* dev[2];
    };
    std::vector<G32> groups;
    bool rebuild32 = true;
    int graph_m = -1;
    drop_graph(b);
    for (;;) {
        // FP64 residual sweep and defect of every active problem
        std::vector<double> host(2 * n, 0.0);
        hipError_t e = hipSuccess;
        for (size_t i = 0; i < n && e == hipSuccess; ++i) {
            if (!b->active[i]) continue;
            thiim_ctx* c = b->ctx[i];
            e = one_pass(c, c->cur, 1 - c->cur);
            if (e == hipSuccess)
                e = thiim::launch_defect(c->F[c->cur], c->F[1 - c->cur], c->r32, c->cv.P, c->L.S,
                                         c->L.N, (long long)c->g.nx * c->g.ny, c->part,
                                         kResidBlocks, c->out, b->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(&host[2 * i], c->out, 2 * sizeof(double),
                                   hipMemcpyDeviceToHost, b->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch mixed: residual");
        bool any = false, weak = false;
        for (size_t i = 0; i < n; ++i) {
            if (!b->active[i]) continue;
            thiim_ctx* c = b->ctx[i];
            done[i] += 1;
            r[i] = std::sqrt(host[2 * i]) / (c->phi0_norm > 0 ? c->phi0_norm : 1.0);
            const bool grew = !std::isfinite(r[i]) || r[i] > kGrowth * best[i];
            if (grew) diverged = true;
            best[i] = std::min(best[i], r[i]);
            if (grew || r[i] <= tol || done[i] >= max_it) {
                b->active[i] = 0;
                rebuild32 = true;
                continue;
            }
            any = true;
            if (std::isfinite(prev[i]) && r[i] > kWeak * prev[i]) weak = true;
        }
        if (!any) break;
        if (m_user <= 0 && weak && m < kMaxInner) m *= 2;
        if (rebuild32) {
            drop_graph(b);
            groups.clear();
            for (size_t i = 0; i < n; ++i) {
                if (!b->active[i]) continue;
                auto it = std::find_if(groups.begin(), groups.end(),
                                       [&](const G32& gr) { return gr.T == T[i]; });
                if (it == groups.end()) {
                    groups.push_back(G32{T[i], {}, 0, {nullptr, nullptr}});
                    it = groups.end() - 1;
                }
                it->members.push_back((int)i);
            }
            std::vector<thiim::BatchItem32> items;
            for (auto& gr : groups) {
                for (int par = 0; par < 2; ++par) {
                    gr.dev[par] = base + items.size();
                    int t = 0;
                    for (int i : gr.members) {
                        thiim_ctx* c = b->ctx[i];
                        thiim::BatchItem32 it;
                        it.ce = c->ce32;
                        it.P32 = c->p32;
                        it.r = c->r32;
                        it.S = c->L.S;
                        it.ph = make_float2((float)c->cv.K.ph.x, (float)c->cv.K.ph.y);
                        it.phc = make_float2((float)c->cv.K.phc.x, (float)c->cv.K.phc.y);
                        it.ph2 = make_float2((float)c->cv.K.ph2.x, (float)c->cv.K.ph2.y);
                        it.ph2c = make_float2((float)c->cv.K.ph2c.x, (float)c->cv.K.ph2c.y);
                        it.A = c->d32[par];
                        it.B = c->d32[1 - par];
                        it.rT = c->rt32;
                        it.acc = c->acc32;
                        it.window = Kp[i];
                        it.g = c->geo;
                        it.kchunk = c->inner_chunk;
                        const int ox = 32 - 2 * gr.T;
                        const int oy = thiim::batch_inner_ry(gr.T) - 2 * gr.T;
                        it.ntx = (c->g.nx + ox - 1) / ox;
                        it.nty = (c->g.ny + oy - 1) / oy;
                        it.ntz = (c->g.nz + it.kchunk - 1) / it.kchunk;
                        it.tile_begin = t;
                        t += it.ntx * it.nty * it.ntz;
                        items.push_back(it);
                    }
                    gr.total = t;
                }
            }
            e = hipMemcpyAsync(base, items.data(), items.size() * sizeof(thiim::BatchItem32),
                               hipMemcpyHostToDevice, b->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
            if (e != hipSuccess) return hip_fail(e, "batch mixed: item upload");
            rebuild32 = false;
        }
        // complex64 inner phase (graph-captured when the stream allows)
        auto inner = [&]() {
            hipError_t err = hipSuccess;
            for (auto& gr : groups) {
                int P = 0;
                for (int i : gr.members) {
                    const int pi = std::max((m - 1 + gr.T - 1) / gr.T, Kp[i]);
                    P = std::max(P, pi);
                }
                for (int i : gr.members) {
                    if (err == hipSuccess) err = launch_rt(b->ctx[i], b->stream);
                    if (err == hipSuccess)
                        err = thiim::launch_copy32(b->ctx[i]->r32, b->ctx[i]->d32[0],
                                                   b->ctx[i]->L.S, b->ctx[i]->L.N, b->stream);
                }
                // each item sums its last Kp passes into its acc32
                int wmax = 0;
                for (int i : gr.members) wmax = std::max(wmax, Kp[i]);
                for (int p = 0; err == hipSuccess && p < P; ++p)
                    err = thiim::launch_inner32_batch(gr.dev[p & 1], (int)gr.members.size(),
                                                      gr.total, gr.T, P - 1 - p, wmax, b->queue,
                                                      b->ncu, b->stream);
                for (int i : gr.members) {
                    if (err != hipSuccess) break;
                    thiim_ctx* c = b->ctx[i];
                    err = thiim::launch_accum(c->F[c->cur], c->acc32, 1.0 / Kp[i], c->cv.P,
                                              0.5, (long long)c->g.nx * c->g.ny, c->L.S,
                                              c->L.N, b->stream);
                }
            }
            return err;
        };
        if (b->stream) {
            if (!b->exec || graph_m != m) {
                drop_graph(b);
                e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) return hip_fail(e, "batch mixed: begin capture");
                hipError_t el = inner();
                e = hipStreamEndCapture(b->stream, &b->graph);
                if (el != hipSuccess) return hip_fail(el, "batch mixed: captured launch");
                if (e != hipSuccess) return hip_fail(e, "batch mixed: end capture");
                e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
                if (e != hipSuccess) return hip_fail(e, "batch mixed: instantiate");
                graph_m = m;
            }
            e = hipGraphLaunch(b->exec, b->stream);
        } else {
            e = inner();
        }
        if (e != hipSuccess) return hip_fail(e, "batch mixed: inner passes");
        for (auto& gr : groups) {
            int P = 0;
            for (int i : gr.members) P = std::max(P, std::max((m - 1 + gr.T - 1) / gr.T, Kp[i]));
            for (int i : gr.members) {
                done[i] += P * gr.T;
                b->ctx[i]->iters += 1 + P * gr.T;
                prev[i] = r[i];
            }
        }
    }
    drop_graph(b);
    return THIIM_OK;
}

}  // namespace

extern "C" {

int thiim_batch_workspace_bytes(int n, size_t* bytes) {
    if (n < 1 || !bytes) return fail(THIIM_EINVAL, "need n >= 1 and bytes");
    *bytes = batch_bytes(n);
    return THIIM_OK;
}

}  // extern "C"

namespace {

int check_batch_contexts(thiim_ctx* const* ctxs, int n) {
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return fail(THIIM_EINVAL, "a context is NULL");
        if (!ctxs[i]->cv.compact) return fail(THIIM_EINVAL, "batches need the compact storage");
        if (ctxs[i]->stream != ctxs[0]->stream)
            return fail(THIIM_EINVAL, "all contexts of a batch must use one stream");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(THIIM_EINVAL, "a context appears twice");
    }
    return THIIM_OK;
}

int make_batch(thiim_ctx* const* ctxs, int n, char* ws, size_t ws_bytes, int static_dev,
               thiim_batch** out) {
    thiim_batch* b = new (std::nothrow) thiim_batch();
    if (!b) return fail(THIIM_EINVAL, "out of host memory");
    b->ctx.assign(ctxs, ctxs + n);
    b->stream = ctxs[0]->stream;
    b->ws = ws;
    b->ws_bytes = ws_bytes;
    b->queue = batch_queue(b, n);
    b->ncu = ctxs[0]->ncu;
    b->active.assign(n, 1);
    b->dirty = true;
    b->graph = nullptr;
    b->exec = nullptr;
    b->graph_iters = kGraphIters;
    b->static_dev = static_dev;
    const hipError_t e = thiim::launch_queue_reset(b->queue, b->stream);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch: queue reset");
    }
    *out = b;
    return THIIM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free batches.  The item tables and queue counters of a batch
// created by thiim_batch_create_static live in `scratch`, a file-scope
// device array of kStaticBatchBytes (room for kStaticBatchMax problems); each
// device holds its own copy until the process ends.  In host code `scratch`
// names a host-side stand-in, so its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that
// address is used (item uploads, kernel arguments).  One static batch per
// device at a time: the scratch keeps the last batch's tables, and a second
// batch would overwrite them, so creation is refused while one is alive.
// ---------------------------------------------------------------------------
constexpr int kStaticBatchMax = 128;
constexpr size_t kStaticBatchBytes = 256 * 1024;
static_assert(batch_bytes(kStaticBatchMax) <= kStaticBatchBytes,
              "static batch scratch too small for kStaticBatchMax problems");

}  // namespace

static __device__ __align__(256) char scratch[kStaticBatchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device
bool g_scratch_busy[kMaxDevices];  // a static batch holds the device's scratch

}  // namespace

extern "C" {

int thiim_batch_create(thiim_ctx* const* ctxs, int n, void* workspace, size_t workspace_bytes,
                       thiim_batch** out) {
    if (!out) return fail(THIIM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctxs || n < 1) return fail(THIIM_EINVAL, "need n >= 1 contexts");
    if (!workspace || (uintptr_t)workspace % kAlign)
        return fail(THIIM_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (workspace_bytes < batch_bytes(n))
        return fail(THIIM_ENOMEM, "workspace smaller than thiim_batch_workspace_bytes()");
    int rc = check_batch_contexts(ctxs, n);
    if (rc) return rc;
    return make_batch(ctxs, n, (char*)workspace, workspace_bytes, -1, out);
}

int thiim_batch_create_static(thiim_ctx* const* ctxs, int n, thiim_batch** out) {
    if (!out) return fail(THIIM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctxs || n < 1) return fail(THIIM_EINVAL, "need n >= 1 contexts");
    if (n > kStaticBatchMax)
        return fail(THIIM_EINVAL, "thiim_batch_create_static: at most " +
                                      std::to_string(kStaticBatchMax) +
                                      " problems (static scratch); use thiim_batch_create");
    int rc = check_batch_contexts(ctxs, n);
    if (rc) return rc;
    const int dev = ctxs[0]->device;
    for (int i = 1; i < n; ++i)
        if (ctxs[i]->device != dev)
            return fail(THIIM_EINVAL, "all contexts of a batch must be on one device");
    if (dev < 0 || dev >= kMaxDevices) return fail(THIIM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_busy[dev])
        return fail(THIIM_EINVAL, "the static batch scratch of this device is held by another "
                                  "batch (destroy it first)");
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void* ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "thiim_batch_create_static: scratch address");
        if (!ptr || (uintptr_t)ptr % kAlign)
            return fail(THIIM_EDEVICE, "thiim_batch_create_static: unaligned scratch");
        g_scratch_ptr[dev] = (char*)ptr;
    }
    rc = make_batch(ctxs, n, g_scratch_ptr[dev], kStaticBatchBytes, dev, out);
    if (rc == THIIM_OK) g_scratch_busy[dev] = true;
    return rc;
}

int thiim_batch_iterate(thiim_batch* b, int n) {
    if (!b || n < 0) return fail(THIIM_EINVAL, "batch is NULL or n < 0");
    return batch_iterate(b, n);
}

int thiim_batch_residual(thiim_batch* b, double* rel_res) {
    if (!b || !rel_res) return fail(THIIM_EINVAL, "batch / rel_res is NULL");
    std::vector<double> r;
    int rc = batch_residual(b, r);
    if (rc) return rc;
    for (size_t i = 0; i < r.size(); ++i) rel_res[i] = r[i];
    return THIIM_OK;
}

int thiim_batch_solve(thiim_batch* b, double tol, int max_it, int check_every, int* iters,
                      double* rel_res) {
    if (!b) return fail(THIIM_EINVAL, "batch is NULL");
    const bool mixed0 = b->ctx[0]->g.precision == THIIM_PRECISION_MIXED;
    if (!(tol > 0.0) || max_it < 0 || check_every < (mixed0 ? 0 : 1))
        return fail(THIIM_EINVAL, "need tol > 0, max_it >= 0, check_every >= 1 (>= 0 MIXED)");
    const size_t n = b->ctx.size();
    std::fill(b->active.begin(), b->active.end(), 1);
    b->dirty = true;
    std::vector<double> r(n, INFINITY), best(n, INFINITY);
    std::vector<int> done(n, 0);
    int step_done = 0, rc = THIIM_OK;
    bool diverged = false;
    int mixed = 0;
    for (size_t i = 0; i < n; ++i) mixed += b->ctx[i]->g.precision == THIIM_PRECISION_MIXED;
    if (mixed && mixed != (int)n)
        return fail(THIIM_EINVAL, "batch solve: contexts mix FP64 and MIXED precision");
    if (mixed) rc = batch_solve_mixed(b, tol, max_it, check_every, done, r, diverged);
    for (; !mixed;) {
        std::vector<double> now;
        rc = batch_residual(b, now);
        if (rc) break;
        bool any = false;
        for (size_t i = 0; i < n; ++i) {
            if (!b->active[i]) continue;
            r[i] = now[i];
            done[i] = step_done;
            const bool grew = !std::isfinite(r[i]) || r[i] > kGrowth * best[i];
            if (grew) diverged = true;
            best[i] = std::min(best[i], r[i]);
            if (grew || r[i] <= tol) {
                b->active[i] = 0;
                b->dirty = true;
            } else {
                any = true;
            }
        }
        if (!any || step_done >= max_it) break;
        const int step = check_every < max_it - step_done ? check_every : max_it - step_done;
        rc = batch_iterate(b, step);
        if (rc) break;
        step_done += step;
    }
    std::fill(b->active.begin(), b->active.end(), 1);
    b->dirty = true;
    for (size_t i = 0; i < n; ++i) {
        if (iters) iters[i] = done[i];
        if (rel_res) rel_res[i] = r[i];
    }
    if (rc) return rc;
    if (diverged)
        return fail(THIIM_EDIVERGED, "batch: a residual is not finite or grew 1e6-fold");
    for (size_t i = 0; i < n; ++i)
        if (!(r[i] <= tol)) return fail(THIIM_ENOTCONV, "batch: iteration limit reached");
    return THIIM_OK;
}

int thiim_batch_autotune(thiim_batch* b, int trial_iters, thiim_tuning* out) {
    if (!b || trial_iters < 1) return fail(THIIM_EINVAL, "batch is NULL or trial_iters < 1");
    struct Cfg {
        int kernel, tx, ty, chunk;  // chunk 0: each problem's automatic chunk
    };
    std::vector<Cfg> cands;
    const int regions[3][2] = {{32, 16}, {64, 8}, {64, 6}};
    for (auto& r : regions)
        for (int zc : {0, 32, 64}) cands.push_back({THIIM_KERNEL_BLOCKED, r[0], r[1], zc});
    for (int zc : {0, 32}) {
        cands.push_back({THIIM_KERNEL_FUSED, 64, 8, zc});
        cands.push_back({THIIM_KERNEL_FUSED, 32, 8, zc});
    }
    auto apply_all = [&](const Cfg& k) {
        for (thiim_ctx* c : b->ctx) {
            const int ox = k.kernel == THIIM_KERNEL_BLOCKED ? k.tx - 4 : k.tx;
            const int oy = k.kernel == THIIM_KERNEL_BLOCKED ? k.ty - 4 : k.ty;
            const long long tiles = (long long)((c->g.nx + ox - 1) / ox) * ((c->g.ny + oy - 1) / oy);
            int zc = k.chunk > 0 ? std::min(k.chunk, c->g.nz) : auto_chunk(c->g, tiles, c->ncu);
            apply(c, Candidate{k.kernel, k.tx, k.ty, zc, 0.0});
        }
        b->dirty = true;
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(THIIM_EDEVICE, "batch autotune: event create");
    // Time of one iteration of every problem under the current assignment:
    // rounds of two iterations each (one pass of each blocked group, two of
    // each fused group), from the current states into the spare buffers (the
    // states do not advance).
    auto time_current = [&](double* per_it) {
        int rc2 = rebuild(b);
        if (rc2) return rc2;
        auto round = [&]() {
            hipError_t e = hipSuccess;
            for (auto& gr : b->groups) {
                for (int rep = 0; rep < (gr.blocked ? 1 : 2) && e == hipSuccess; ++rep)
                    e = gr.blocked
                            ? thiim::launch_blocked_batch(gr.dev[gr.par], (int)gr.members.size(),
                                                          gr.total, 2, gr.tx, gr.ty, b->queue,
                                                          b->ncu, b->stream)
                            : thiim::launch_fused_batch(gr.dev[gr.par], (int)gr.members.size(),
                                                        gr.total, gr.tx, gr.ty, b->queue,
                                                        b->ncu, b->stream);
            }
            return e;
        };
        const int rounds = (trial_iters + 1) / 2;
        hipError_t e = round();
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        for (int p = 0; e == hipSuccess && p < rounds; ++p) e = round();
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) return hip_fail(e, "batch autotune trial");
        *per_it = ms / (2.0 * rounds);
        return THIIM_OK;
    };
    // one configuration for every problem
    int best = -1;
    double best_ms = INFINITY;
    int rc = THIIM_OK;
    for (size_t i = 0; i < cands.size() && rc == THIIM_OK; ++i) {
        apply_all(cands[i]);
        double per_it = INFINITY;
        rc = time_current(&per_it);
        if (rc == THIIM_OK && per_it < best_ms) {
            best_ms = per_it;
            best = (int)i;
        }
    }
    // per grid: each distinct grid shape takes the choice of thiim_autotune on
    // one of its problems alone, then the batch is timed with that mix
    double grid_ms = INFINITY;
    std::vector<Candidate> grid_cfg(b->ctx.size());
    for (size_t i = 0; i < b->ctx.size() && rc == THIIM_OK; ++i) {
        const thiim_grid& gi = b->ctx[i]->g;
        size_t j = 0;
        while (j < i && !(b->ctx[j]->g.nx == gi.nx && b->ctx[j]->g.ny == gi.ny &&
                          b->ctx[j]->g.nz == gi.nz))
            ++j;
        if (j < i) {
            grid_cfg[i] = grid_cfg[j];
            continue;
        }
        thiim_tuning t;
        rc = thiim_autotune(b->ctx[i], trial_iters, &t);
        grid_cfg[i] = Candidate{t.kernel, t.tile_x, t.tile_y, t.z_chunk, 0.0};
    }
    if (rc == THIIM_OK) {
        for (size_t i = 0; i < b->ctx.size(); ++i) apply(b->ctx[i], grid_cfg[i]);
        b->dirty = true;
        rc = time_current(&grid_ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (best < 0) return fail(THIIM_EDEVICE, "batch autotune: no trial produced a timing");
    const bool per_grid = grid_ms < best_ms;
    if (per_grid) {
        for (size_t i = 0; i < b->ctx.size(); ++i) apply(b->ctx[i], grid_cfg[i]);
        b->dirty = true;
    } else {
        apply_all(cands[best]);
    }
    if (out) {
        out->kernel = cands[best].kernel;
        out->tile_x = cands[best].tx;
        out->tile_y = cands[best].ty;
        out->t_block = cands[best].kernel == THIIM_KERNEL_BLOCKED ? 2 : 1;
        out->z_chunk = cands[best].chunk;
        out->ms_per_iteration = per_grid ? grid_ms : best_ms;
        out->model_ms = 0.0;
        out->candidates = (int)cands.size() + 1;
        out->timed = (int)cands.size() + 1;
        out->one_for_all_ms = best_ms;
        out->per_grid_ms = grid_ms;
        out->per_grid = per_grid ? 1 : 0;
    }
    return THIIM_OK;
}

void thiim_batch_destroy(thiim_batch* b) {
    if (!b) return;
    drop_graph(b);
    if (b->static_dev >= 0) {
        // no kernel of this batch may still read the tables when the next
        // static batch overwrites them
        (void)hipStreamSynchronize(b->stream);
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        g_scratch_busy[b->static_dev] = false;
    }
    delete b;
}

int thiim_stream_probe(const double* src, double* dst, long long n, long long stride, int nin,
                       int nout, void* stream) {
    if (!src || !dst || n < 1 || stride < n)
        return fail(THIIM_EINVAL, "stream probe: need src, dst, n >= 1 and stride >= n");
    if (!((nin == 1 && nout == 1) || (nin == 13 && nout == 12)))
        return fail(THIIM_EINVAL, "stream probe: (nin, nout) must be (1, 1) or (13, 12)");
    if (n * 16 > 0xFFFFFFFFLL) return fail(THIIM_EINVAL, "stream probe: arrays must be < 4 GiB");
    if ((uintptr_t)src % 16 || (uintptr_t)dst % 16)
        return fail(THIIM_EINVAL, "stream probe: buffers must be 16-byte aligned");
    hipError_t e = thiim::launch_stream_probe((const double2*)src, (double2*)dst, stride, n, nin,
                                              nout, cu_count(), (hipStream_t)stream);
    return e == hipSuccess ? THIIM_OK : hip_fail(e, "stream probe launch");
}

int thiim_iterations(const thiim_ctx* c, long long* n) {
    if (!c || !n) return fail(THIIM_EINVAL, "ctx / n is NULL");
    *n = c->iters;
    return THIIM_OK;
}

void thiim_destroy(thiim_ctx* c) { delete c; }

const char* thiim_last_error(void) { return g_last_error.c_str(); }

const char* thiim_status_str(int s) {
    switch (s) {
        case THIIM_OK: return "THIIM_OK";
        case THIIM_EINVAL: return "THIIM_EINVAL";
        case THIIM_ENOMEM: return "THIIM_ENOMEM";
        case THIIM_EDEVICE: return "THIIM_EDEVICE";
        case THIIM_EDIVERGED: return "THIIM_EDIVERGED";
        case THIIM_ENOTCONV: return "THIIM_ENOTCONV";
        default: return "THIIM_UNKNOWN";
    }
}

}  // extern "C"
