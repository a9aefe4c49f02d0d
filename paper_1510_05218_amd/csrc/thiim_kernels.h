// Internal interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace thiim {

struct Geo {
    int nx, ny, nz;
    int bcx, bcy;  // 0 periodic, 1 Dirichlet
    long long S;   // stride between arrays (double2 elements)
};

// Constants of the coefficient formulas (Eq. 3-5).
struct CoefConst {
    double tau, h, omega;
    double2 ph, phc, ph2, ph2c;  // e^{iwt}, e^{-iwt}, e^{iwt/2}, e^{-iwt/2}
};

// Per-plane coefficient data (96 bytes).  H coefficients depend only on the
// plane: sigma* = 0 on the x/y-difference parts, sigma_h(z) on H_xy, H_yx.
struct PlaneCoef {
    double2 th0, thz;  // t of H parts without / with the PML term
    double2 ch0, chz;  // c of H parts without / with the PML term
    double2 shz;       // Src scale of H_xy, H_yx (tau / d_H)
    double sig_e;      // electric PML conductivity of E_xy, E_yx
    int has_src;       // a source value on this plane is non-zero
    int pad;
};

// H coefficients of one plane rounded to complex64 (inner sweeps of the
// mixed-precision solver), and which split pairs of the plane have two parts
// with identical coefficients: on such a plane the defect step stores the
// same value for both parts of the pair in r (k_defect_partial), and the
// inner sweeps read it once.
struct PlaneCoef32 {
    float2 th0, thz, ch0, chz;
    int hsym;    // the x and y pairs of H (the z pair always)
    int esym;    // the x and y pairs of E (the z pair always)
    int pad[2];
};

// Where the sweeps find their coefficients.
//   full:    the 28 arrays of the paper's layout (t_q, c_q, 4 Src) at C
//   compact: per-cell eps (1 array) + the 4 Src arrays; t, c derived on the
//            fly by the same device functions that build the full arrays
struct CoefView {
    int compact;
    const double2* C;    // full: 28 arrays
    const double2* eps;  // compact: (eps', eps'') per cell
    const double2* src;  // 4 Src arrays (full: C + 24*S)
    const PlaneCoef* P;  // nz entries
    long long S;
    CoefConst K;
};

// One problem of a batched pass (compact storage, FP64): its coefficient
// view, source / destination buffers, grid, z chunk and its range in the
// concatenated tile list (tile_begin, ntx * nty * ntz tiles).
struct BatchItem {
    CoefView cv;
    const double2* A;
    double2* B;
    Geo g;
    int kchunk;
    int tile_begin;
    int ntx, nty, ntz;
};

// One problem of a batched complex64 inner pass (mixed precision): the
// inner-sweep coefficient data, residual r, d buffers, grid and tile range.
struct BatchItem32 {
    const float4* ce;
    const PlaneCoef32* P32;
    const float2* r;
    long long S;
    float2 ph, phc, ph2, ph2c;
    const float2* A;
    float2* B;
    const float2* rT;  // last-stage source of the two-sweep passes
    float2* acc;  // window sum of the correction (pair-sum form)
    int window;   // passes in the window: the last `window` passes of a step
    Geo g;
    int kchunk;
    int tile_begin;
    int ntx, nty, ntz;
};

struct BuildArgs {
    const double2* eps_in;   // (eps', eps'') per cell
    const double* sig_e;     // nz, device
    const double* sig_h;     // nz, device
    const double2* src_in[4];  // S_Hx, S_Hy, S_Ex, S_Ey or null
    double2* C;              // full: 28 arrays (else null)
    double2* eps_out;        // compact: copy of eps (else null)
    double2* src_out;        // 4 Src arrays
    PlaneCoef* P;            // nz entries
    long long S, N, nxy;
    int nz;
    CoefConst K;
    int* flag;               // set to 1 on invalid material data
};

hipError_t launch_build(const BuildArgs& a, bool compact, hipStream_t s);
hipError_t launch_expand(const CoefView& cv, const Geo& g, double2* dst, hipStream_t s);
hipError_t launch_naive(const CoefView& cv, double2* F, const Geo& g, int kchunk,
                        hipStream_t s);
hipError_t launch_fused(const CoefView& cv, const double2* A, double2* B, const Geo& g,
                        int tile_x, int tile_y, int kchunk, hipStream_t s);
// The fused pass A -> B that also writes r2 = ||P(B - A)||^2 and b2 = ||P B||^2
// (physical components, FP64) to out[0], out[1]: one partial pair per
// workgroup in part (at most max_blocks workgroups; the z chunking is
// coarsened to fit), summed in a fixed order.
hipError_t launch_fused_res(const CoefView& cv, const double2* A, double2* B, const Geo& g,
                            int tile_x, int tile_y, int kchunk, double* part, int max_blocks,
                            double* out, hipStream_t s);
hipError_t launch_blocked(const CoefView& cv, const double2* A, double2* B, const Geo& g,
                          int T, int rx, int ry, int kchunk, hipStream_t s);
// Mixed precision: the per-cell complex64 E-coefficient records and the
// per-plane H table (once per context), then inner sweeps d <- M d + r.
hipError_t launch_prep32(const CoefView& cv, const Geo& g, float4* ce, PlaneCoef32* P32,
                         hipStream_t s);
// One complex64 inner pass of T sweeps d <- M d + r (T = 2 on 32 x 32 regions,
// T = 3 on 32 x 16), or with src_last (T = 2) d <- M^T d + r with r added at
// the last stage only (r then holds r_T = (I + M) r of the sweep source),
// adding the stored d to acc with acc_mode 1 (acc = d) or 2 (acc += d).
hipError_t launch_inner32(const CoefView& cv, const float4* ce, const PlaneCoef32* P32,
                          const float2* r, bool src_last, const float2* A, float2* B,
                          float2* acc, int acc_mode, const Geo& g, int T, int rx, int ry,
                          int kchunk, hipStream_t s);
hipError_t launch_defect(const double2* A, const double2* B, float2* R, const PlaneCoef* P,
                         long long S, long long N, long long nxy, double* part, int nblk,
                         double* out, hipStream_t s);
// x += w d; with a plane table P (nxy cells per plane) a symmetric pair of d
// is stored as its first part and each part of the pair receives share * w
// times it (1/2: the pair-sum form of the forward inner sweeps, 1: the
// pair-equal form of the transposed ones); P = nullptr: d holds all 12 parts
hipError_t launch_accum(double2* X, const float2* D, double w, const PlaneCoef* P,
                        double share, long long nxy, long long S, long long N, hipStream_t s);
hipError_t launch_copy32(const float2* src, float2* dst, long long S, long long N,
                         hipStream_t s);
// Batched passes over nitems problems whose tiles total `total` (items in
// device memory, ordered by tile_begin): persistent launches of at most the
// resident workgroups (ncu CUs) that take tiles from a device work queue of
// 9 counters at `queue` (zero before the first pass, see launch_queue_reset;
// every pass leaves them zero again; launches sharing a queue must be ordered
// on one stream).
// Zeroes the counters of a batch's device work queue (once, when the batch is
// made: every persistent pass leaves them zero for the next).
hipError_t launch_queue_reset(unsigned int* queue, hipStream_t s);
hipError_t launch_fused_batch(const BatchItem* items, int nitems, int total, int tile_x,
                              int tile_y, unsigned int* queue, int ncu, hipStream_t s);
hipError_t launch_blocked_batch(const BatchItem* items, int nitems, int total, int T, int rx,
                                int ry, unsigned int* queue, int ncu, hipStream_t s);
// Regions of the batched inner passes: 32 x 24 for two sweeps per pass,
// 32 x 16 for three.
constexpr int batch_inner_ry(int T) { return T == 2 ? 24 : 16; }
// left: passes of the step after this one (an item sums its last `window`);
// max_window: the largest window of the items
hipError_t launch_inner32_batch(const BatchItem32* items, int nitems, int total, int T, int left,
                                int max_window, unsigned int* queue, int ncu, hipStream_t s);
// ||P(B - A)||^2 and ||P B||^2 over the physical components c0..5 (0: all
// six, 3: E only) into out[0], out[1].
hipError_t launch_resid(const double2* A, const double2* B, long long S, long long N,
                        int c0, double* part, int nblk, double* out, hipStream_t s);
// Adjoint (compact storage): one transposed iteration A -> B with source G
// (3 arrays); the objective / adjoint source of the state X (J in out[0]);
// the gradient (dJ/deps', dJ/deps'') per cell.
hipError_t launch_adjoint(const CoefView& cv, const double2* A, double2* B, const double2* G,
                          bool dense, const Geo& g, int tile_x, int tile_y, int kchunk,
                          hipStream_t s);
// Complex64 transposed sweep with a 12-array source R (inner sweeps of the
// adjoint defect correction on mixed-precision contexts).
hipError_t launch_adjoint32(const CoefView& cv, const float4* ce, const PlaneCoef32* P32,
                            const float2* A, float2* B, const float2* R, const Geo& g,
                            int tile_x, int tile_y, int kchunk, hipStream_t s);
// T = 2 transposed iterations per pass (regions of 32 x 16 columns) of the
// same complex64 sweep; chunk planes per workgroup stream
// acc_mode 1 writes the pass's output also to acc, 2 adds it to acc (12
// complex64 arrays), 0 leaves acc alone.  Regions 32 x 16 with the source R
// at every stage (src_last false), or 32 x 24 at three waves per SIMD with R
// = G_T = (I + M^T) G entering at the last stage only (src_last true).
hipError_t launch_adjoint32_blocked(const CoefView& cv, const float4* ce, const PlaneCoef32* P32,
                                    const float2* A, float2* B, const float2* R, bool src_last,
                                    float2* acc, int acc_mode, const Geo& g, int T, int rx,
                                    int ry, int kchunk, hipStream_t s);
// 12-array FP64 helpers: Y -= X; X += w D.
hipError_t launch_sub(const double2* X, double2* Y, long long S, long long N, hipStream_t s);
hipError_t launch_to32(const double2* X, float2* R, long long S, long long N, hipStream_t s);
hipError_t launch_axpy(double2* X, const double2* D, double w, long long S, long long N,
                       hipStream_t s);
hipError_t launch_adj_source(const double2* X, const double2* eps, const double* w, long long S,
                             long long N, double2* G, double* part, int nblk, double* out,
                             hipStream_t s);
hipError_t launch_adj_grad(const CoefView& cv, const double2* X, const double2* Y,
                           const double2* L, const double* w, const Geo& g, double2* grad,
                           hipStream_t s);
hipError_t launch_stream_probe(const double2* in, double2* out, long long S, long long n,
                               int nin, int nout, int ncu, hipStream_t s);
hipError_t launch_fill_zero(double2* p, long long n, hipStream_t s);
hipError_t launch_copy(const double2* src, double2* dst, long long n, hipStream_t s);

}  // namespace thiim
