// Internal interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace thiim {

struct Geo {
    int nx, ny, nz;
    int bcx, bcy;  // 0 periodic, 1 Dirichlet
    long long S;   // stride between arrays (double2 elements)
};

struct CoefArgs {
    const double2* eps;      // (eps', eps'') per cell
    const double* sig_e;     // nz, device
    const double* sig_h;     // nz, device
    const double2* src[4];   // S_Hx, S_Hy, S_Ex, S_Ey or null
    double2* coef;           // 28 arrays, stride S
    long long S, N, nxy;
    double tau, h, omega;
    double2 ph, phc, ph2, ph2c;  // e^{iwt}, e^{-iwt}, e^{iwt/2}, e^{-iwt/2}
    int* flag;               // set to 1 on invalid material data
};

hipError_t launch_coeffs(const CoefArgs& a, hipStream_t s);
hipError_t launch_naive(const double2* C, double2* F, const Geo& g, int kchunk,
                        hipStream_t s);
hipError_t launch_fused(const double2* C, const double2* A, double2* B, const Geo& g,
                        int tile_x, int tile_y, int kchunk, hipStream_t s);
hipError_t launch_blocked(const double2* C, const double2* A, double2* B, const Geo& g,
                          int T, int ry, int kchunk, hipStream_t s);
hipError_t launch_resid(const double2* A, const double2* B, long long S, long long N,
                        double* part, int nblk, double* out, hipStream_t s);
hipError_t launch_fill_zero(double2* p, long long n, hipStream_t s);
hipError_t launch_copy(const double2* src, double2* dst, long long n, hipStream_t s);

}  // namespace thiim
